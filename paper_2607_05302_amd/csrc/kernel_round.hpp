// One digit round of Radsort's sortPhase (Alg. 5) on the GPU, and the
// out-of-place round of Alg. 1 built from the same tile code.
//
// A tile is E consecutive element slots of the logical block sequence
// sigma .. f-1 (slot s of logical block L holds element s if s < len(L)).  How
// workgroups take tiles is the launch form (below); in every form a tile waits
// only on lower tiles, and the lowest unfinished tile is being worked on with all
// of its predecessors finished, so the waits always end.  Tiles come in
// super-tiles of 2^st_log2; a pass before the kernel gives the digit counts
// before every super-tile (kernels_prefix.hpp).
//
//   1  read the tile's blocks through pi (keys and payload) into registers (with
//      PF, while the workgroup still works on its previous tile);
//   2  stable rank inside the tile, per wave: for each group of 64 slots, every
//      lane ORs its lane bit into a wave-private LDS word of its digit and reads
//      the word back, which gives the lanes holding the same digit; lower lanes
//      of that set come first (slot order).  Per-wave digit counts in LDS;
//   3  publish the tile's digit counts, and stage the tile in LDS in (digit,
//      slot) order;
//   4  a decoupled look-back over the earlier tiles of the super-tile (up to
//      kLookbackWin per step, so usually one step) plus the super-tile's start
//      gives base[d], the number of digit-d elements before the tile.  A
//      look-back over all earlier tiles would chain every tile of the launch to
//      the one before it;
//   5  global rank r = base[d] + local rank.  Bucket d's block q holds ranks
//      [q b, (q+1) b) and sits at logical index S[d] + q (Alg. 6).  Block q >= 1
//      is drawn when rank q b - 1 is written (eager allocation, Alg. 5).  Blocks
//      are drawn from the pool pi_old[0..] in input order, as the sequential
//      algorithm draws them: the first blocks of the buckets are pool entries
//      0..sigma-1, block draws number sigma, sigma+1, ....  A tile finds its
//      draws' pool indices from base[] (draws in earlier tiles are
//      F = sum_d floor(base[d]/b)) plus its rank among the tile's own draws: in
//      (digit, block) order by default, in slot order (the sequential order)
//      with SEQ; it publishes pi_new[S[d] + q] for each draw.  A bucket's block that holds
//      the tile's first elements of that digit was drawn by an earlier tile: its
//      pi_new entry is requested as soon as base[] is known and waited for only
//      after the tile's own draws are out (waiting first would chain each tile
//      to the draws of the one before);
//   6  write each element to blockat(pi_new[S[d] + q]) + (r mod b).
//
// Why a drawn block is never overwritten before it is read (the GPU form of
// Lemma 1): draws up to tile k number at most sum_d floor(ranks_d / b) <=
// floor(E_k / b), with E_k the elements of tiles <= k, and these tiles cover at
// least ceil(E_k / b) logical blocks, so every drawn pool index names a
// head-start block or an input block of a tile <= k.  A tile publishes its counts
// only after its loads returned; before publishing its draws (later tiles write
// into a drawn block as soon as they see its entry) a tile waits for the counts
// of their tiles (those of its own super-tile it has already read in the
// look-back) or for their done word.
//
// P and f after every round are those of the sequential algorithm, and so is pi
// with SEQ; the default order permutes the pool entries within each tile.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace rs {

constexpr int kLookbackWin = 16;  // predecessors read per look-back step

// Look-back words.  cnt[slot][d] holds a tile's count of digit d in bits 0-30
// and, in bit 31, the parity of the tile's ring epoch (floor(tile / W)) inverted,
// so that the zero-filled array reads as "not yet" for epoch 0.  (16-bit words
// would halve the look-back's reads, but measured slower on MI355X.)  done[slot] holds
// tile + 1 once the tile has finished its look-back.  Slot = tile mod W.
//
// A slot is reused by tile T only after every tile of the super-tile of T - W,
// from T - W on, is done: those are the only readers of its counts, and T - W
// published before it was done.  So a reader of a predecessor's slot finds
// either that tile's word or the one before it (W tiles earlier), and the parity
// bit tells them apart.  done[] only grows within a slot, so done[o mod W] > o
// says that tile o is done, hence that its loads have returned.
constexpr uint32_t kCntMask = 0x7FFFFFFFu;
__device__ __forceinline__ uint32_t epoch_bit(uint32_t tile, uint32_t wlog)
{
    return (~(tile >> wlog) & 1u) << 31;
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
    uint32_t* agg;           // tile counts [2^ring_log2][sigma], zeroed per round
    uint32_t* done;          // [2^ring_log2]: tile + 1 once done, zeroed per round
    const uint32_t* stbase;  // [super-tile][sigma]: digit counts before each super-tile
    uint32_t* err;
    uint32_t* tile_ctr;      // dynamic launches: next tile to claim, zero on entry
    uint32_t shift, bits, log2b, npi, ring_log2;
    uint32_t st_log2;        // tiles per super-tile: 2^st_log2
    uint64_t* tl;            // timeline builds only: kTlStamps stamps per tile, or null
    uint32_t* consumed;      // ordering-check builds only: per physical block, the tag of
    uint32_t tag;            // the round whose loads of it returned last; or null
    uint32_t tag_mark;       // the tag the marks carry (differs only to test the check)
    // The packed round (the last before finalize; null / npi otherwise): bucket d
    // starts at offset est[d] mod b of its head block (plan_round), and the pool of
    // draws is sigma extra blocks X (physical npi .. npi + sigma - 1) followed by
    // the input blocks in logical order, which keeps every draw behind the blocks
    // already read although the offsets make buckets draw up to sigma blocks early.
    const uint32_t* pack_est;
    K* Xk;
    V* Xv;
    uint32_t npi_x;          // physical blocks a draw can name: npi, + sigma when packed
};

// Timeline builds (RS_TIMELINE defined): thread 0 of each workgroup records the
// 100 MHz real-time counter at the phase boundaries of every tile, so that a
// profiling run can attribute the round's time to its steps.  Normal builds
// record nothing.
constexpr int kTlStamps = 16;
#ifdef RS_TIMELINE
#define RS_STAMP(k)                                                                       \
    do {                                                                                  \
        if (threadIdx.x == 0 && a.tl)                                                     \
            a.tl[(uint64_t)tile * kTlStamps + (k)] = __builtin_amdgcn_s_memrealtime();    \
    } while (0)
#else
#define RS_STAMP(k) \
    do {            \
    } while (0)
#endif


// Three launch forms (DYN).  kPersistent: a cooperative launch of as many
// workgroups as are resident, each taking tiles in grid-stride order.  kPerTile:
// one workgroup per tile, launched normally, each claiming its tile from a
// counter; a tile is claimed only by a running workgroup, so every lower tile is
// already claimed by one and the waits still end.  kClaimLoop: a normal launch of
// at most as many workgroups as fit, each claiming its next tile from the counter
// while it works on the current one; a workgroup finishes its lower tile first, so
// the lowest unfinished tile is always being worked on and depends only on finished
// ones.  The last two need no co-residency, so several sorts can share the GPU, and
// they save the cooperative launch of every round: measured alone, kPerTile is the
// faster Radsort round for blocks of up to 1024 elements and kClaimLoop the faster
// out-of-place round.
constexpr int kPersistent = 0, kPerTile = 1, kClaimLoop = 2;

// Shape of a round's workgroup (see TileCfg in radsort.hip): WAVES waves of 64
// lanes with ITEMS slots each; PF: the next tile's records are loaded into
// registers while the current tile is processed (for one workgroup per CU);
// SPLIT: the payload is staged in LDS only after the keys have been scattered,
// in the same LDS, which halves the staging area so that more workgroups fit on
// a CU; OCC: waves per SIMD the register allocation must allow.
template <int WAVES_, int ITEMS_, bool PF_, bool SPLIT_, int OCC_> struct RoundShape {
    static constexpr int WAVES = WAVES_, ITEMS = ITEMS_, OCC = OCC_;
    static constexpr bool PF = PF_, SPLIT = SPLIT_;
};

// SEQ: a tile's draws take their pool entries in the slot order of the elements
// that fill the blocks, as the sequential scan of Alg. 5 does, so that pi after
// every round equals the sequential algorithm's.  Otherwise in (digit, block)
// order: each tile still draws the same pool entries, only their assignment to
// the tile's filled blocks differs, and the slot of every staged element need
// not be kept.
template <int KB, int VB, bool OOP, int FB, int SMAX, class SH, int DYN = kPersistent,
          bool SEQ = true>
__global__ __launch_bounds__(SH::WAVES * 64)
__attribute__((amdgpu_waves_per_eu(SH::OCC))) void k_round(TileArgs<KB, VB> a)
{
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    constexpr int WAVES = SH::WAVES, ITEMS = SH::ITEMS;
    constexpr bool PF = SH::PF;
    constexpr bool OR_RANK_ = SMAX <= 256;
    constexpr bool SPLIT = SH::SPLIT && VB != 0 && OR_RANK_;  // two-pass staging
    constexpr int NT = WAVES * 64;
    constexpr int E = NT * ITEMS;
    constexpr int SEG = E / WAVES;
    constexpr int MAXBLK = E / 64;
    constexpr int TBL = MAXBLK + 2 * SMAX;        // blocks one tile can write
    constexpr bool OR_RANK = SMAX <= 256;         // OR-table ranking fits in LDS
    constexpr int PTAB = OR_RANK ? 4 * TBL : 0;  // words of the pointer table
    constexpr int LSW = SEQ ? E / 2 : 0;          // words of the slot array
    constexpr int UNI = (LSW + 2 * SMAX) > PTAB ? (LSW + 2 * SMAX) : PTAB;
    static_assert(E <= 65536, "slot indices are 16-bit");
    static_assert((E & (E - 1)) == 0, "tiles and super-tiles are powers of two");
    static_assert(WAVES >= 4, "per-digit scratch reuses the per-wave counts");
    static_assert(!OR_RANK || E * KB >= WAVES * SMAX * 8, "OR tables live in the key stage");

    const uint32_t bits = FB ? (uint32_t)FB : a.bits;
    const uint32_t sigma = 1u << bits, dmask = sigma - 1;
    const uint32_t log2b = a.log2b, b = 1u << log2b, two_sigma = 2 * sigma;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // keys in (digit, slot) order (OR tables before); with SPLIT the payload
    // follows in the same bytes once the keys are written out
    constexpr int SB = SPLIT ? (KB > VB ? KB : VB) : KB;
    __shared__ __align__(16) unsigned char stage[E * SB];
    K* lk = (K*)stage;
    __shared__ V lv_[(VB && !SPLIT) ? E : 1];    // payload in the same order (no SPLIT)
    V* lv = SPLIT ? (V*)stage : lv_;
    __shared__ __align__(16) uint32_t uni[UNI];  // slots + cnt + excl, later the pointer table
    __shared__ __align__(16) uint32_t wh[WAVES * SMAX];  // per-wave counts, later per-digit data
    // EARLY: the tile's draws are published before it is staged, and the entries of
    // the blocks drawn by earlier tiles are waited for after staging, which covers
    // the time those tiles' publications take to become visible.  The per-digit
    // data then needs its own arrays (staging still reads the wave offsets).
    constexpr bool EARLY = !SEQ && !OOP;
    __shared__ uint32_t pd_base[EARLY ? SMAX : 1], pd_nfw[EARLY ? SMAX : 1];
    __shared__ uint2 pd_dt[EARLY ? SMAX : 1];
    __shared__ uint32_t tbo[SMAX];
    __shared__ uint32_t tphys[TBL];
    __shared__ uint32_t pool[OOP ? 1 : TBL];     // physical blocks of the tile's draws
    __shared__ uint32_t fmask[SEQ ? E / 32 : 1], fpref[SEQ ? E / 32 : 1];
    __shared__ uint32_t fbo[SEQ ? 1 : SMAX];     // first draw of each digit (digit order)
    __shared__ uint32_t bphys[MAXBLK], blen[MAXBLK];
    __shared__ uint32_t tmp[3 * (NT / 64) + 2];

    uint16_t* ls = (uint16_t*)uni;               // slot of each staged element (SEQ)
    uint32_t* cnt = uni + LSW;
    uint32_t* excl = uni + LSW + SMAX;

    const uint32_t wlog = a.ring_log2;
    const uint64_t wmask = (1ull << wlog) - 1;
    const uint32_t mst = 1u << a.st_log2;  // tiles per super-tile
    // f is clamped so that a corrupt state can never index past pi
    const uint32_t f_in = OOP ? 0u : max(sigma, min(*a.f_in, a.npi));
    uint64_t nslots;
    if constexpr (OOP) nslots = a.n;
    else nslots = (uint64_t)(f_in - sigma) << log2b;
    const uint32_t ntiles = (uint32_t)((nslots + E - 1) / E);

    // physical index and used length of the blocks of a tile: loaded into
    // registers (thread i < blocks per tile holds block i), then put in bphys / blen
    static_assert(MAXBLK <= NT, "one thread per block of a tile");
    const uint32_t nblk = (E >> log2b) ? (E >> log2b) : 1u;
    auto block_info_load = [&](uint32_t t, uint32_t& phys, uint32_t& len) {
        phys = 0;
        len = 0;
        if constexpr (!OOP) {
            const uint32_t L = sigma + (uint32_t)(((uint64_t)t * E) >> log2b) + tid;
            if (tid < nblk && L < f_in) {
                phys = a.pi_old[L];
                len = min(a.blen[L], b);
            }
        }
    };
    auto block_info_store = [&](uint32_t phys, uint32_t len) {
        if constexpr (!OOP) {
            if (tid < nblk) {
                if (phys >= a.npi) {  // never for a consistent state; read nothing
                    raise_error(a.err, kErrBounds);
                    phys = 0;
                    len = 0;
                }
                bphys[tid] = phys;
                blen[tid] = len;
            }
        }
    };
    // issue the loads of tile t into (kn, vn); block info of t must be in LDS
    K kn[ITEMS];
    V vn[ITEMS];
    bool vld[ITEMS];
    auto load_tile = [&](uint32_t t) {
        const uint64_t slot0 = (uint64_t)t * E;
        const uint32_t blk0 = (uint32_t)(slot0 >> log2b);
        if constexpr (!OOP) {
            if (b >= (uint32_t)SEG) {
                // the wave's SEG slots lie in one block: one table lookup, then
                // loads at fixed offsets from one base
                const uint64_t ws0 = slot0 + wave * SEG;
                const uint32_t bi = (uint32_t)(ws0 >> log2b) - blk0;
                const uint32_t off0 = (uint32_t)ws0 & (b - 1);
                const uint32_t len = t < ntiles ? blen[bi] : 0u;
                const uint32_t phys = t < ntiles ? bphys[bi] : 0u;
                const K* kb = blockat(a.Ak, a.Tk, phys, two_sigma, log2b) + off0 + lane;
                const V* vb = nullptr;
                if constexpr (VB != 0) vb = blockat(a.Av, a.Tv, phys, two_sigma, log2b) + off0 + lane;
#pragma unroll
                for (int j = 0; j < ITEMS; j++) {
                    const bool valid = off0 + j * 64 + lane < len;
                    vld[j] = valid;
                    kn[j] = valid ? kb[j * 64] : (K)0;
                    if constexpr (VB != 0) vn[j] = valid ? vb[j * 64] : (V)0;
                }
                return;
            }
        }
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            const uint64_t gs = slot0 + wave * SEG + j * 64 + lane;
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
                valid = t < ntiles && off < blen[bi];
                const uint32_t phys = bphys[bi];
                kp = blockat(a.Ak, a.Tk, phys, two_sigma, log2b) + off;
                if constexpr (VB != 0) vp = blockat(a.Av, a.Tv, phys, two_sigma, log2b) + off;
            }
            vld[j] = valid;
            kn[j] = valid ? *kp : (K)0;
            if constexpr (VB != 0) vn[j] = valid ? *vp : (V)0;
        }
    };
    uint32_t first_tile = blockIdx.x;
#ifdef RS_TIMELINE
    const uint64_t t_entry = __builtin_amdgcn_s_memrealtime();
#endif
    __shared__ uint32_t claimed;  // the tile claimed next (claimed forms)
    if constexpr (DYN != kPersistent) {
        if (tid == 0) claimed = add_agent(a.tile_ctr, 1u);
        __syncthreads();
        first_tile = claimed;
    }
    {
        uint32_t phys, len;
        block_info_load(first_tile, phys, len);
        block_info_store(phys, len);
    }
    __syncthreads();
    if constexpr (PF) load_tile(first_tile);

    for (uint32_t tile = first_tile, next; tile < ntiles; tile = next) {
#ifdef RS_TIMELINE
    if (tile == first_tile && tid == 0 && a.tl)
        a.tl[(uint64_t)tile * kTlStamps + 15] = t_entry;
#endif
    RS_STAMP(0);
    // without PF the tile's loads are issued here; its block info is in LDS
    if constexpr (!PF) load_tile(tile);
    K key[ITEMS];
    V val[ITEMS];
    uint32_t rk[ITEMS];  // wave-local rank << 12 | digit, or ~0 for an empty slot
    bool allv = true;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        key[j] = kn[j];
        if constexpr (VB != 0) val[j] = vn[j];
        rk[j] = vld[j] ? 0u : ~0u;
        allv = allv && vld[j];
    }
    // every slot of the wave holds an element (all but a few waves of a round):
    // the per-item checks below are left out
    const bool wfull = ballot(!allv) == 0;
    if constexpr (DYN == kClaimLoop) {  // the next tile, one ahead: its loads overlap this one
        if (tid == 0) claimed = add_agent(a.tile_ctr, 1u);
    }
    __syncthreads();  // the previous tile is done with LDS
    next = DYN == kClaimLoop ? claimed : DYN == kPerTile ? ntiles : tile + gridDim.x;
    for (uint32_t i = lane; i < SMAX; i += 64) wh[wave * SMAX + i] = 0;
    if constexpr (OR_RANK) {
        uint64_t* myor = (uint64_t*)lk + wave * SMAX;
        for (uint32_t i = lane; i < SMAX; i += 64) myor[i] = 0;
    }
    // the next tile's block info: loaded now, put in LDS when this tile is staged
    // (its loads are issued after that)
    uint32_t nx_phys, nx_len;
    block_info_load(next, nx_phys, nx_len);

    // Reuse of this tile's ring slot (see the look-back words above): the done
    // words of the tiles that must have finished are requested now and checked
    // before this tile publishes its counts; those tiles started W tiles earlier,
    // so the check almost never polls twice.
    uint32_t rq = 0, rqend = 0, rv = 0;
    if ((uint64_t)tile > wmask) {
        rq = tile - (uint32_t)wmask - 1;                    // tile - W
        rqend = min((rq | (mst - 1)) + 1, ntiles);          // end of its super-tile
        if (rq + tid < rqend) rv = ld_agent(a.done + ((rq + tid) & wmask));
    }

    // ---- stable rank among equal digits of the wave ----------------------------------
    uint32_t* myh = wh + wave * SMAX;
    if constexpr (OR_RANK) {
        uint64_t* myor = (uint64_t*)lk + wave * SMAX;
        const uint64_t mybit = 1ull << lane;
        auto or_rank = [&](auto full) {
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                if (full.value || rk[j] != ~0u) {
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
        };
        if (wfull) or_rank(std::true_type{});
        else or_rank(std::false_type{});
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
    // Every load of the tile has returned (the payload is not read before staging,
    // so wait for it here): from the counts' publication on, other tiles may
    // reuse the tile's blocks.
    for (uint32_t j = rq + tid; j < rqend; j += NT) {
        const uint32_t* w = a.done + (j & wmask);
        uint32_t v = j == rq + tid ? rv : ld_agent(w), spins = 0;
        while (v <= j) {
            if (spin_give_up(++spins, a.err)) break;
            spin_pause();
            v = ld_agent(w);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    RS_STAMP(1);
#ifdef RS_DEBUG_ORDER
    // Ordering check: the tile's input blocks are marked as read (every load has
    // returned), and the marks are released before the counts that allow the
    // blocks' reuse.  Empty blocks (a bucket whose count is a multiple of b ends in
    // one) are marked too: they hold nothing to read.  A block spans several tiles
    // when b > E: checked only for b <= E.
    if constexpr (!OOP) {
        if (a.consumed && b <= (uint32_t)E) {
            const uint32_t L = sigma + (uint32_t)(((uint64_t)tile * E) >> log2b) + tid;
            if (tid < nblk && L < f_in) st_agent(a.consumed + bphys[tid], a.tag_mark);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
        }
    }
#endif

    // ---- per-digit tile counts (published at once) and wave offsets ------------------
    const uint32_t st0 = tile & ~(mst - 1);  // first tile of this tile's super-tile
    uint32_t* mycnt = a.agg + (uint64_t)(tile & wmask) * sigma;
    uint32_t total;
    if constexpr (SMAX <= NT) {
        // one digit per thread: its count, the scan over the digits and the wave
        // offsets in one pass
        const uint32_t d = tid;
        uint32_t run = 0;
        if (d < sigma) {
#pragma unroll
            for (int w = 0; w < WAVES; w++) {
                const uint32_t c = wh[w * SMAX + d];
                wh[w * SMAX + d] = run;
                run += c;
            }
            st_agent(mycnt + d, run | epoch_bit(tile, wlog));
            cnt[d] = run;
        }
        const uint32_t incl = wave_incl_scan(run);
        if (lane == 63) tmp[wave] = incl;
        __syncthreads();
        uint32_t before = 0;
        total = 0;
#pragma unroll
        for (uint32_t w = 0; w < NT / 64; w++) {
            const uint32_t t = tmp[w];
            before += w < wave ? t : 0u;
            total += t;
        }
        if (d < sigma) {
            const uint32_t ex = before + incl - run;
            excl[d] = ex;
#pragma unroll
            for (int w = 0; w < WAVES; w++) wh[w * SMAX + d] += ex;
        }
    } else {
        for (uint32_t d = tid; d < sigma; d += NT) {
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < WAVES; w++) {
                const uint32_t c = wh[w * SMAX + d];
                wh[w * SMAX + d] = run;
                run += c;
            }
            st_agent(mycnt + d, run | epoch_bit(tile, wlog));
            cnt[d] = run;
            excl[d] = run;
        }
        __syncthreads();
        total = block_excl_scan<NT>(excl, sigma, tmp);
        for (uint32_t d = tid; d < sigma; d += NT) {
#pragma unroll
            for (int w = 0; w < WAVES; w++) wh[w * SMAX + d] += excl[d];
        }
    }
    __syncthreads();
    RS_STAMP(2);

    // ---- stage in (digit, slot) order ------------------------------------------------
    // (with SPLIT, rk[j] keeps the staged position for the payload pass)
    auto stage_tile = [&]() {
    RS_STAMP(13);
    auto stage_items = [&](auto full) {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            if (full.value || rk[j] != ~0u) {
                const uint32_t d = rk[j] & 0xFFFu;
                const uint32_t p = wh[wave * SMAX + d] + (rk[j] >> 12);
                lk[p] = key[j];
                if constexpr (VB != 0 && !SPLIT) lv[p] = val[j];
                if constexpr (SEQ) ls[p] = (uint16_t)(wave * SEG + j * 64 + lane);
                if constexpr (SPLIT) rk[j] = p;
            }
        }
    };
    if (wfull) stage_items(std::true_type{});
    else stage_items(std::false_type{});
    block_info_store(nx_phys, nx_len);
    __syncthreads();
    RS_STAMP(3);
    // registers are free again: issue the next tile's loads
    if constexpr (PF) load_tile(next);
    };
    if constexpr (!EARLY) stage_tile();

    // per-digit data (reusing the wave counts once the tile is staged)
    uint32_t* base = EARLY ? pd_base : wh;
    uint32_t* nfw = EARLY ? pd_nfw : wh + SMAX;
    uint2* dt = EARLY ? pd_dt : (uint2*)(wh + 2 * SMAX);  // (rank offset, table offset)

    // ---- look back over the super-tile -----------------------------------------------
    for (uint32_t d = tid; d < sigma; d += NT) {
        // the super-tile's digit start, requested with the first look-back loads
        const uint32_t sbase = a.stbase[(uint64_t)(tile >> a.st_log2) * sigma + d];
        // sum the counts of tiles st0 .. tile-1, up to kLookbackWin loads at once;
        // while one has not published, poll that one alone
        uint32_t acc = 0, k = tile, spins = 0;
        bool stalled = false;
        while (k > st0) {
            const uint32_t m = stalled ? 1u : min<uint32_t>(kLookbackWin, k - st0);
            uint32_t w[kLookbackWin];
#pragma unroll
            for (int i = 0; i < kLookbackWin; i++)
                if ((uint32_t)i < m)
                    w[i] = ld_agent(a.agg + (uint64_t)((k - 1 - i) & wmask) * sigma + d);
            uint32_t used = 0;
            bool ready = true;
#pragma unroll
            for (int i = 0; i < kLookbackWin; i++) {
                if ((uint32_t)i < m && ready) {
                    if ((w[i] & ~kCntMask) == epoch_bit(k - 1 - i, wlog)) {
                        acc += w[i] & kCntMask;
                        used = i + 1;
                    } else {
                        ready = false;
                    }
                }
            }
            k -= used;
            stalled = !ready && used == 0;
            if (!ready) {
                if (spin_give_up(++spins, a.err)) break;
                spin_pause();
            }
        }
        base[d] = sbase + acc;
        if constexpr (!OOP)
            if (a.pack_est) base[d] += a.pack_est[d] & (b - 1);  // the packed round's offset
    }
    __syncthreads();
    RS_STAMP(4);
    if (tid == 0) st_agent(a.done + (tile & wmask), tile + 1);

    if constexpr (OOP) {
        for (uint32_t d = tid; d < sigma; d += NT) dt[d].x = a.est[d] + base[d] - excl[d];
        __syncthreads();
        if constexpr (SPLIT) {
            // keys first, remembering each position's destination; then the
            // payload is staged in the same LDS and written to the same places
            uint32_t dst[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                const uint32_t p = tid + i * NT;
                dst[i] = ~0u;
                if (p < total) {
                    const K k = lk[p];
                    const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
                    const uint64_t pos = (uint64_t)p + dt[d].x;
                    if (pos < a.n) {
                        a.Tk[pos] = k;
                        dst[i] = (uint32_t)pos;
                    } else {  // never for consistent digit starts
                        raise_error(a.err, kErrBounds);
                    }
                }
            }
            __syncthreads();  // every staged key was read
#pragma unroll
            for (int j = 0; j < ITEMS; j++)
                if (rk[j] != ~0u) lv[rk[j]] = val[j];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                const uint32_t p = tid + i * NT;
                if (dst[i] != ~0u) a.Tv[dst[i]] = lv[p];
            }
        } else {
            for (uint32_t p = tid; p < total; p += NT) {
                const K k = lk[p];
                const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
                const uint64_t pos = (uint64_t)p + dt[d].x;
                if (pos < a.n) {
                    a.Tk[pos] = k;
                    if constexpr (VB != 0) a.Tv[pos] = lv[p];
                } else {  // never for consistent digit starts
                    raise_error(a.err, kErrBounds);
                }
            }
        }
    } else {
        // ---- block draws ----------------------------------------------------------------
        // the block a draw names: Eq. 1, or one of the packed round's extra blocks
        auto out_block = [&](auto* A, auto* T, auto* X, uint32_t j) {
            return j < a.npi ? blockat(A, T, j, two_sigma, log2b)
                             : X + ((uint64_t)(j - a.npi) << log2b);
        };
        // Request the block that takes each digit's first elements (drawn by an
        // earlier tile) now; it is used after this tile's own draws are out.
        uint32_t first = kEmpty;  // pi_new entry of that block, for digit tid
        uint32_t fsum = 0, nsum = 0, wsum = 0;
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t bs = base[d], c = cnt[d], q0 = bs >> log2b;
            const uint32_t nfill = ((bs + c) >> log2b) - q0;
            const uint32_t nwrite = c ? ((bs + c - 1) >> log2b) - q0 + 1 : 0u;
            const uint32_t L = a.S[d] + q0;
            if (d == tid && c && q0 > 0 && L < a.npi_x) first = ld_agent(a.pi_new + L);
            nfw[d] = (nfill << 16) | nwrite;
            tbo[d] = nwrite;
            if constexpr (!SEQ) fbo[d] = nfill;
            fsum += q0;
            nsum += nfill;
            wsum += nwrite;
        }
        if constexpr (SEQ)
            for (uint32_t i = tid; i < E / 32; i += NT) fmask[i] = 0;
        // F: draws made by earlier tiles; nfills: draws of this tile; with one
        // digit per thread, also the scans of the blocks each digit writes and
        // (digit order) of the blocks it draws
        const uint32_t myfill = nsum;
        const uint32_t fincl = (!SEQ && SMAX <= NT) ? wave_incl_scan(myfill) : 0u;
        fsum = wave_sum(fsum);
        nsum = wave_sum(nsum);
        const uint32_t wincl = SMAX <= NT ? wave_incl_scan(wsum) : 0u;
        if (lane == 0) {
            tmp[wave] = fsum;
            tmp[NT / 64 + wave] = nsum;
        }
        if (SMAX <= NT && lane == 63) tmp[2 * (NT / 64) + wave] = wincl;
        __syncthreads();
        uint32_t F = 0, nfills = 0, wbefore = 0, nent = 0, fbefore = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; w++) {
            F += tmp[w];
            const uint32_t tf = tmp[NT / 64 + w];
            nfills += tf;
            fbefore += (uint32_t)w < wave ? tf : 0u;
            if constexpr (SMAX <= NT) {
                const uint32_t t = tmp[2 * (NT / 64) + w];
                wbefore += (uint32_t)w < wave ? t : 0u;
                nent += t;
            }
        }
        RS_STAMP(10);
        if constexpr (SMAX <= NT) {
            if (tid < sigma) {
                tbo[tid] = wbefore + wincl - wsum;
                if constexpr (!SEQ) fbo[tid] = fbefore + fincl - myfill;
            }
        }
        // request the pool entries of the draws, and the done words of the
        // earlier tiles whose input blocks they are.  Draw k of the round takes pool
        // entry k: the input block sigma + k (logical), or in the packed round the
        // extra block npi + k for k < sigma and then the input block k.
        const bool packed = a.pack_est != nullptr;
        auto pool_entry = [&](uint32_t k) -> uint32_t {
            if (packed) return k < sigma ? a.npi + k : (k < a.npi ? a.pi_old[k] : a.npi_x);
            const uint32_t h = sigma + k;
            return h < a.npi ? a.pi_old[h] : a.npi_x;
        };
        uint32_t pv = 0;
        if (tid < nfills) pv = pool_entry(F + tid);
        // input blocks (counted from the round's first) among the drawn entries
        const uint32_t in_lo = packed ? (F > sigma ? F - sigma : 0u) : F;
        const uint32_t in_hi = packed ? (F + nfills > sigma ? F + nfills - sigma : 0u) : F + nfills;
        uint32_t olo = 0, ohi = 0, dv = ~0u;
        if (in_hi > in_lo) {
            olo = (uint32_t)(((uint64_t)in_lo << log2b) / E);
            ohi = min<uint32_t>((uint32_t)((((uint64_t)in_hi << log2b) - 1) / E) + 1, st0);
            if (olo + tid < ohi) dv = ld_agent(a.done + ((olo + tid) & wmask));
        }
        if constexpr (SMAX > NT) {
            __syncthreads();  // tmp is reused by the scans
            nent = block_excl_scan<NT>(tbo, sigma, tmp);
            if constexpr (!SEQ) block_excl_scan<NT>(fbo, sigma, tmp);
        }
        // mark the slots whose element fills a block
        if constexpr (SEQ) {
            for (uint32_t d = tid; d < sigma; d += NT) {
                const uint32_t nfill = nfw[d] >> 16, bs = base[d], q0 = bs >> log2b;
                for (uint32_t i = 1; i <= nfill; i++) {
                    const uint32_t lr = ((q0 + i) << log2b) - 1 - bs;
                    const uint32_t s = ls[excl[d] + lr];
                    atomicOr(&fmask[s >> 5], 1u << (s & 31));
                }
            }
        }
        // The drawn blocks are input blocks sigma + F .. sigma + F + nfills - 1.  Those
        // of this super-tile were loaded before their tiles' counts, which the
        // look-back read; for earlier tiles wait until they are done.  The wait ends
        // before the draws are published (after the barrier below): later tiles
        // that continue a drawn block write into it as soon as they see its entry
        // in pi_new, and they make no wait of their own for its old contents.
        for (uint32_t o = olo + tid; o < ohi; o += NT) {
            const uint32_t* w = a.done + (o & wmask);
            uint32_t v = o == olo + tid ? dv : ld_agent(w), spins = 0;
            while (v <= o) {
                if (spin_give_up(++spins, a.err)) break;
                spin_pause();
                v = ld_agent(w);
            }
        }
        if constexpr (SEQ) {
            __syncthreads();
            for (uint32_t i = tid; i < E / 32; i += NT) fpref[i] = __popc(fmask[i]);
        }
        if (tid < nfills) pool[tid] = pv;
        for (uint32_t i = tid + NT; i < nfills; i += NT)  // more draws than threads: rare
            pool[i] = pool_entry(F + i);
        __syncthreads();
        RS_STAMP(11);
#ifdef RS_DEBUG_ORDER
        // Ordering check: every drawn block that holds input of this round (pool
        // entry below f) must be marked read by its tile before the draw is
        // published; the waits above (or the look-back, for this super-tile) ordered it.
        if (a.consumed && b <= (uint32_t)E) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (uint32_t i = tid; i < nfills; i += NT) {
                const uint32_t phys = pool[i];
                if (sigma + F + i < f_in && phys < a.npi && ld_agent(a.consumed + phys) != a.tag)
                    raise_error(a.err, kErrOrder);
            }
        }
#endif
        if constexpr (SEQ) block_excl_scan<NT>(fpref, E / 32, tmp);
        // publish the tile's draws for every digit
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t bs = base[d], q0 = bs >> log2b;
            const uint32_t nfill = nfw[d] >> 16, nwrite = nfw[d] & 0xFFFFu, t0 = tbo[d];
            const uint32_t Sd = a.S[d];
            for (uint32_t i = 1; i <= nfill; i++) {
                uint32_t r;  // the draw's rank among the tile's draws
                if constexpr (SEQ) {
                    const uint32_t lr = ((q0 + i) << log2b) - 1 - bs;
                    const uint32_t s = ls[excl[d] + lr];
                    r = fpref[s >> 5] + __popc(fmask[s >> 5] & ((1u << (s & 31)) - 1u));
                } else {
                    r = fbo[d] + i - 1;
                }
                const uint32_t L = Sd + q0 + i;
                uint32_t phys = r < nfills ? pool[r] : a.npi_x;
                if (phys < a.npi_x && L < a.npi_x) {
                    st_agent(a.pi_new + L, phys);
                } else {
                    raise_error(a.err, kErrBounds);
                    phys = 0;
                }
                if (i < nwrite) tphys[t0 + i] = phys;
            }
        }
        RS_STAMP(12);
        if constexpr (EARLY) stage_tile();
        // the block of each digit's first elements
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t bs = base[d], c = cnt[d], q0 = bs >> log2b;
            if (c) {
                uint32_t phys = d == tid ? first : kEmpty;
                if (q0 == 0) {
                    phys = a.pi_old[d];
                } else if (a.S[d] + q0 >= a.npi_x) {
                    raise_error(a.err, kErrBounds);
                    phys = 0;
                } else {
                    uint32_t spins = 0;
                    while (phys == kEmpty) {
                        if (spin_give_up(++spins, a.err)) { phys = 0; break; }
                        spin_pause();
                        phys = ld_agent(a.pi_new + a.S[d] + q0);
                    }
                }
                tphys[tbo[d]] = phys;
            }
            dt[d] = make_uint2(bs - excl[d], tbo[d] - q0);
        }
        __syncthreads();
        RS_STAMP(5);
        for (uint32_t e = tid; e < nent; e += NT) {
            if (tphys[e] >= a.npi_x) {  // never for a consistent state: send the writes to T
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
                ptab[2 * e] = (uint64_t)(uintptr_t)out_block(a.Ak, a.Tk, a.Xk, j);
                if constexpr (VB != 0)
                    ptab[2 * e + 1] = (uint64_t)(uintptr_t)out_block(a.Av, a.Tv, a.Xv, j);
            }
            __syncthreads();
            RS_STAMP(6);
            // ---- scatter ------------------------------------------------------------
            if constexpr (SPLIT) {
                // keys first, remembering (table entry, offset) of each position;
                // then the payload is staged in the same LDS and follows its key
                uint32_t dst[ITEMS];
                const bool tfull = total == (uint32_t)E;  // the same for the workgroup
                auto scatter_keys = [&](auto full) {
#pragma unroll
                    for (int i = 0; i < ITEMS; i++) {
                        const uint32_t p = tid + i * NT;
                        dst[i] = ~0u;
                        if (full.value || p < total) {
                            const K k = lk[p];
                            const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
                            const uint2 x = dt[d];
                            const uint32_t r = p + x.x;
                            const uint32_t e = x.y + (r >> log2b);
                            const uint32_t off = r & (b - 1);
                            st_global((K*)(uintptr_t)ptab[2 * e] + off, k);
                            dst[i] = e << 16 | off;  // e < TBL < 2^16, off < b <= 2^16
                        }
                    }
                };
                if (tfull) scatter_keys(std::true_type{});
                else scatter_keys(std::false_type{});
                __syncthreads();  // every staged key was read
                RS_STAMP(7);
                if (wfull) {
#pragma unroll
                    for (int j = 0; j < ITEMS; j++) lv[rk[j]] = val[j];
                } else {
#pragma unroll
                    for (int j = 0; j < ITEMS; j++)
                        if (rk[j] != ~0u) lv[rk[j]] = val[j];
                }
                __syncthreads();
                RS_STAMP(8);
                auto scatter_vals = [&](auto full) {
#pragma unroll
                    for (int i = 0; i < ITEMS; i++) {
                        const uint32_t p = tid + i * NT;
                        if (full.value || dst[i] != ~0u)
                            st_global((V*)(uintptr_t)ptab[2 * (dst[i] >> 16) + 1] +
                                          (dst[i] & 0xFFFFu),
                                      lv[p]);
                    }
                };
                if (tfull) scatter_vals(std::true_type{});
                else scatter_vals(std::false_type{});
                __builtin_amdgcn_s_waitcnt(0);
                RS_STAMP(9);
            } else {
                for (uint32_t p = tid; p < total; p += NT) {
                    const K k = lk[p];
                    const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
                    const uint2 x = dt[d];
                    const uint32_t r = p + x.x;
                    const uint32_t e = x.y + (r >> log2b);
                    const uint32_t off = r & (b - 1);
                    st_global((K*)(uintptr_t)ptab[2 * e] + off, k);
                    if constexpr (VB != 0) st_global((V*)(uintptr_t)ptab[2 * e + 1] + off, lv[p]);
                }
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
                out_block(a.Ak, a.Tk, a.Xk, j)[off] = k;
                if constexpr (VB != 0) out_block(a.Av, a.Tv, a.Xv, j)[off] = lv[p];
            }
        }
    }
    }  // tiles
}

}  // namespace rs
