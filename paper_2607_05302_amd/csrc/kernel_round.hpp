// One digit round of Radsort's sortPhase (Alg. 5) on the GPU, and the
// out-of-place round of Alg. 1 built from the same tile code.
//
// A tile is E consecutive element slots of the logical block sequence
// sigma .. f-1 (slot s of logical block L holds element s if s < len(L)).  The
// kernel is persistent and launched cooperatively, so all its workgroups are
// resident at once; workgroup w takes tiles w, w + G, w + 2G, ... (G workgroups).
// A tile waits only on lower tiles, and the lowest unfinished tile has all of its
// predecessors finished, so the waits always end.  (A shared tile counter would
// serialise the launch on one atomic: about 11 ns per tile on MI355X.)
//
//   1  read the tile's blocks through pi (keys and payload);
//   2  stable rank inside the tile, per wave: for each group of 64 slots, every
//      lane ORs its lane bit into a wave-private LDS word of its digit and reads
//      the word back, which gives the lanes holding the same digit; lower lanes
//      of that set come first (slot order).  Per-wave digit counts in LDS;
//   3  stage the tile in LDS in (digit, slot) order;
//   4  publish the tile's digit counts, then decoupled look-back over earlier
//      tiles (reading up to kLookbackWin predecessors per step) gives base[d],
//      the number of digit-d elements before the tile;
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

constexpr int kLookbackWin = 4;  // predecessors read per look-back step

// 16-bit tile-count words of the look-back: bits 0-12 the tile's count of a digit,
// bit 13 set once the tile's inclusive prefix is in the 64-bit ring, bits 14-15
// the tile's round-local epoch mod 4.  The array is zeroed before each round, so a
// slot holds the epoch before, at or after the one a reader expects: the three are
// told apart mod 4.  Reading these words instead of 64-bit ones cuts the
// look-back's coherent traffic by four; the 64-bit word is read only once, for
// the nearest tile whose hint bit is set.
constexpr uint32_t kAggHint = 1u << 13;
__device__ __forceinline__ uint16_t ld_agent16(const uint16_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent16(uint16_t* p, uint16_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
    const uint32_t* blen;    // used length of every logical block of the input
    const uint32_t* f_in;    // fill level of the input
    const uint32_t* S;       // first logical block of each output bucket
    uint64_t* opened;        // per bucket: (q << 32 | physical) of its latest drawn block
    const uint32_t* est;     // out-of-place only: element start of each bucket
    uint64_t n;              // out-of-place only
    uint64_t* ring;          // inclusive prefixes [2^ring_log2][sigma]: count | flag | epoch
    uint16_t* agg;           // tile counts [2^ring_log2][sigma]: count | hint | tag, zeroed per round
    uint32_t* err;
    uint64_t seq_base;       // ring sequence number of tile 0 of this round
    uint32_t shift, bits, log2b, npi, ring_log2;
};

__device__ __forceinline__ uint64_t pack_status(uint64_t count, uint64_t flag, uint64_t epoch)
{
    return count | (flag << 32) | (epoch << 34);
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
    constexpr int TBL = MAXBLK + 2 * SMAX;        // blocks one tile can write
    constexpr bool OR_RANK = SMAX <= 256;         // OR-table ranking fits in LDS
    constexpr int PTAB = OR_RANK ? 4 * TBL : 0;  // words of the pointer table
    constexpr int UNI = (E / 2 + 2 * SMAX) > PTAB ? (E / 2 + 2 * SMAX) : PTAB;
    static_assert(E <= 65536, "slot indices are 16-bit");
    static_assert(E < 8192, "tile counts fit the 13-bit field of the look-back words");
    static_assert(WAVES >= 4, "per-digit scratch reuses the per-wave counts");
    static_assert(!OR_RANK || E * KB >= WAVES * SMAX * 8, "OR tables live in the key stage");

    const uint32_t bits = FB ? (uint32_t)FB : a.bits;
    const uint32_t sigma = 1u << bits, dmask = sigma - 1;
    const uint32_t log2b = a.log2b, b = 1u << log2b, two_sigma = 2 * sigma;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    __shared__ K lk[E];                          // keys in (digit, slot) order; OR tables before
    __shared__ V lv[VB ? E : 1];                 // payload in the same order
    __shared__ __align__(16) uint32_t uni[UNI];  // slots + cnt + excl, later the pointer table
    __shared__ __align__(16) uint32_t wh[WAVES * SMAX];  // per-wave counts, later per-digit data
    __shared__ uint32_t tbo[SMAX];
    __shared__ uint32_t tphys[TBL];
    __shared__ uint32_t fmask[E / 32], fpref[E / 32];
    __shared__ uint32_t bphys[MAXBLK], blen[MAXBLK];
    __shared__ uint32_t tmp[NT / 64 + 1];

    uint16_t* ls = (uint16_t*)uni;               // slot of each staged element
    uint32_t* cnt = uni + E / 2;
    uint32_t* excl = uni + E / 2 + SMAX;

    const uint32_t wlog = a.ring_log2;
    const uint64_t wmask = (1ull << wlog) - 1;
    // f is clamped so that a corrupt state can never index past pi
    const uint32_t f_in = OOP ? 0u : max(sigma, min(*a.f_in, a.npi));
    uint64_t nslots;
    if constexpr (OOP) nslots = a.n;
    else nslots = (uint64_t)(f_in - sigma) << log2b;
    const uint32_t ntiles = (uint32_t)((nslots + E - 1) / E);

    // physical index and used length of the blocks of a tile, into bphys / blen
    auto block_info = [&](uint32_t t) {
        if constexpr (!OOP) {
            const uint32_t b0 = (uint32_t)(((uint64_t)t * E) >> log2b);
            const uint32_t nblk = (E >> log2b) ? (E >> log2b) : 1u;
            for (uint32_t i = tid; i < nblk; i += NT) {
                const uint32_t L = sigma + b0 + i;
                uint32_t phys = 0, len = 0;
                if (L < f_in) {
                    phys = a.pi_old[L];
                    len = min(a.blen[L], b);
                    if (phys >= a.npi) {  // never for a consistent state; read nothing
                        raise_error(a.err, kErrBounds);
                        phys = 0;
                        len = 0;
                    }
                }
                bphys[i] = phys;
                blen[i] = len;
            }
        }
    };
    block_info(blockIdx.x);

    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // the previous tile is done with LDS; this tile's block info is in
    for (uint32_t i = lane; i < SMAX; i += 64) wh[wave * SMAX + i] = 0;
    if constexpr (OR_RANK) {
        uint64_t* myor = (uint64_t*)lk + wave * SMAX;
        for (uint32_t i = lane; i < SMAX; i += 64) myor[i] = 0;
    }
    const uint64_t g = a.seq_base + tile;  // ring sequence number of the tile
    const uint64_t slot0 = (uint64_t)tile * E;

    const uint32_t blk0 = (uint32_t)(slot0 >> log2b);

    // ---- load --------------------------------------------------------------------------
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

    // The ring slot of this tile last held tile - W; its readers are done once tile
    // - W + 1 is inclusive (a reader that still meets the old word starts over).
    // That tile started W - 1 tiles earlier, so this wait almost never polls twice.
    // It is checked here so that its latency overlaps the loads.
    if ((uint64_t)tile > wmask) {
        const uint32_t tp = tile - (uint32_t)wmask;  // tile - W + 1
        const uint32_t tag = ((tp >> wlog) + 1) & 3u;
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint16_t* w = a.agg + (uint64_t)(tp & wmask) * sigma + d;
            uint32_t spins = 0;
            for (;;) {
                const uint32_t s = ld_agent16(w);
                const uint32_t t = s >> 14;
                if (t == ((tag + 1) & 3u) || (t == tag && (s & kAggHint))) break;
                if (spin_give_up(++spins, a.err)) break;
                spin_pause();
            }
        }
    }

    // ---- stable rank among equal digits of the wave ----------------------------------
    uint32_t* myh = wh + wave * SMAX;
    if constexpr (OR_RANK) {
        uint64_t* myor = (uint64_t*)lk + wave * SMAX;
        const uint64_t mybit = 1ull << lane;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            if (rk[j] != ~0u) {
                const uint32_t d = (uint32_t)(key[j] >> a.shift) & dmask;
                __hip_atomic_fetch_or(myor + d, mybit, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint64_t peers = myor[d];
                const uint32_t old = myh[d];
                if ((peers >> lane) == 1ull) {  // highest lane of the set: commit
                    myh[d] = old + (uint32_t)__popcll(peers);
                    myor[d] = 0;
                }
                rk[j] = ((old + popc_below(peers)) << 12) | d;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            const bool valid = rk[j] != ~0u;
            const uint32_t d = (uint32_t)(key[j] >> a.shift) & dmask;
            uint64_t peers = ballot(valid);
            for (uint32_t k = 0; k < bits; k++) {
                const bool bit = (d >> k) & 1u;
                const uint64_t bk = ballot(valid && bit);
                peers &= bit ? bk : ~bk;
            }
            if (valid) {
                const uint32_t old = myh[d];
                if ((peers >> lane) == 1ull) myh[d] = old + (uint32_t)__popcll(peers);
                rk[j] = ((old + popc_below(peers)) << 12) | d;
            }
        }
    }
    __syncthreads();
    // every wave has issued its loads: fetch the next tile's block info meanwhile
    block_info(tile + gridDim.x);

    // ---- per-digit tile counts, wave offsets and the tile's digit starts -------------
    for (uint32_t d = tid; d < sigma; d += NT) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < WAVES; w++) {
            const uint32_t c = wh[w * SMAX + d];
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

    // ---- stage in (digit, slot) order ------------------------------------------------
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

    uint32_t* base = wh;                  // per-digit data reusing the wave counts
    uint32_t* nfw = wh + SMAX;
    uint2* dt = (uint2*)(wh + 2 * SMAX);  // (rank offset, table offset) per digit

    // ---- publish counts and look back ------------------------------------------------
    {
        const uint64_t ep = (g >> wlog) + 1;                  // epoch of the 64-bit ring
        const uint32_t mytag = ((tile >> wlog) + 1) & 3u;     // round-local epoch mod 4
        uint64_t* myinc = a.ring + (g & wmask) * sigma;
        uint16_t* myagg = a.agg + (uint64_t)(tile & wmask) * sigma;
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t c = cnt[d];
            uint64_t acc = 0;
            if (tile == 0) {
                st_agent(myinc + d, pack_status(c, kFlagInc, ep));
                st_agent16(myagg + d, (uint16_t)(c | kAggHint | (mytag << 14)));
            } else {
                st_agent16(myagg + d, (uint16_t)(c | (mytag << 14)));
                uint32_t k = tile;  // predecessors not yet summed: tiles 0 .. k-1
                uint32_t spins = 0;
                bool stalled = false;  // the nearest predecessor had nothing published yet
                for (;;) {
                    // read up to kLookbackWin predecessors at once; while waiting for
                    // one that has not published, poll that one alone
                    const uint32_t m = stalled ? 1u : min<uint32_t>(kLookbackWin, k);
                    uint32_t w[kLookbackWin];
#pragma unroll
                    for (int i = 0; i < kLookbackWin; i++) {
                        if ((uint32_t)i < m)
                            w[i] = ld_agent16(a.agg + (uint64_t)((k - 1 - i) & wmask) * sigma + d);
                    }
                    uint32_t used = 0;
                    int state = 0;  // 0: all summed, 1: hint found, 2: not ready, 3: restart
#pragma unroll
                    for (int i = 0; i < kLookbackWin; i++) {
                        if ((uint32_t)i < m && state == 0) {
                            const uint32_t want = (((k - 1 - i) >> wlog) + 1) & 3u;
                            const uint32_t t = w[i] >> 14;
                            if (t == want) {
                                used = i + 1;
                                if (w[i] & kAggHint) state = 1;
                                else acc += w[i] & 0x1FFFu;
                            } else if (t == ((want + 1) & 3u)) {
                                state = 3;
                            } else {
                                state = 2;
                            }
                        }
                    }
                    if (state == 1) {
                        // the nearest tile with an inclusive prefix: read it from the ring
                        const uint64_t gk = a.seq_base + k - used, want = (gk >> wlog) + 1;
                        const uint64_t* p = a.ring + (gk & wmask) * sigma + d;
                        bool ok = false;
                        for (;;) {
                            const uint64_t s = ld_agent(p);
                            if ((s >> 34) == want && ((s >> 32) & 3u) == kFlagInc) {
                                acc += (uint32_t)s;
                                ok = true;
                                break;
                            }
                            if ((s >> 34) > want) break;  // overwritten: start over
                            if (spin_give_up(++spins, a.err)) { ok = true; break; }
                            spin_pause();
                        }
                        if (ok) break;
                        acc = 0;
                        k = tile;
                        stalled = false;
                        continue;
                    }
                    if (state == 3) {  // overwritten by a later tile: start over
                        acc = 0;
                        k = tile;
                        stalled = false;
                        continue;
                    }
                    k -= used;
                    if (k == 0) break;  // never: tile 0 is always inclusive
                    stalled = state == 2 && used == 0;
                    if (state == 2) {
                        if (spin_give_up(++spins, a.err)) break;
                        spin_pause();
                    }
                }
                st_agent(myinc + d, pack_status(acc + c, kFlagInc, ep));
                st_agent16(myagg + d, (uint16_t)(c | kAggHint | (mytag << 14)));
            }
            base[d] = (uint32_t)acc;
        }
    }
    __syncthreads();

    if constexpr (OOP) {
        for (uint32_t d = tid; d < sigma; d += NT) dt[d].x = a.est[d] + base[d] - excl[d];
        __syncthreads();
        for (uint32_t p = tid; p < total; p += NT) {
            const K k = lk[p];
            const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
            const uint64_t pos = (uint64_t)p + dt[d].x;
            a.Tk[pos] = k;
            if constexpr (VB != 0) a.Tv[pos] = lv[p];
        }
    } else {
        // ---- block draws --------------------------------------------------------------
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
        const uint32_t nent = block_excl_scan<NT>(tbo, sigma, tmp);
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
                    __hip_atomic_fetch_max(a.opened + d, ((uint64_t)(q0 + i) << 32) | phys,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    raise_error(a.err, kErrBounds);
                }
                if (i < nwrite) tphys[t0 + i] = phys;
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
                    // drawn by an earlier tile.  Usually it is the bucket's latest draw,
                    // read from one coalesced word per bucket; otherwise wait for its
                    // entry of pi'.
                    const uint64_t o = ld_agent(a.opened + d);
                    if ((uint32_t)(o >> 32) == q0) {
                        phys = (uint32_t)o;
                    } else {
                        uint32_t spins = 0;
                        for (;;) {
                            phys = ld_agent(a.pi_new + Sd + q0);
                            if (phys != kEmpty) break;
                            if (spin_give_up(++spins, a.err)) { phys = 0; break; }
                            spin_pause();
                        }
                    }
                }
                tphys[t0] = phys;
            }
            dt[d] = make_uint2(bs - excl[d], t0 - q0);
        }
        __syncthreads();
        for (uint32_t e = tid; e < nent; e += NT) {
            if (tphys[e] >= a.npi) {  // never for a consistent state: send the writes to T
                raise_error(a.err, kErrBounds);
                tphys[e] = 0;
            }
        }
        if constexpr (OR_RANK) {
            // pointer table over the slot area, which is no longer read
            __syncthreads();
            uint64_t* ptab = (uint64_t*)uni;
            for (uint32_t e = tid; e < nent; e += NT) {
                const uint32_t j = tphys[e];
                ptab[2 * e] = (uint64_t)(uintptr_t)blockat(a.Ak, a.Tk, j, two_sigma, log2b);
                if constexpr (VB != 0)
                    ptab[2 * e + 1] = (uint64_t)(uintptr_t)blockat(a.Av, a.Tv, j, two_sigma, log2b);
            }
            __syncthreads();
            // ---- scatter ------------------------------------------------------------
            for (uint32_t p = tid; p < total; p += NT) {
                const K k = lk[p];
                const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
                const uint2 x = dt[d];
                const uint32_t r = p + x.x;
                const uint32_t e = x.y + (r >> log2b);
                const uint32_t off = r & (b - 1);
                ((K*)(uintptr_t)ptab[2 * e])[off] = k;
                if constexpr (VB != 0) ((V*)(uintptr_t)ptab[2 * e + 1])[off] = lv[p];
            }
        } else {
            // wide digits: the pointer table would not fit in LDS
            __syncthreads();
            for (uint32_t p = tid; p < total; p += NT) {
                const K k = lk[p];
                const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
                const uint2 x = dt[d];
                const uint32_t r = p + x.x;
                const uint32_t j = tphys[x.y + (r >> log2b)];
                const uint32_t off = r & (b - 1);
                blockat(a.Ak, a.Tk, j, two_sigma, log2b)[off] = k;
                if constexpr (VB != 0) blockat(a.Av, a.Tv, j, two_sigma, log2b)[off] = lv[p];
            }
        }
    }
    }  // tiles
}

}  // namespace rs
