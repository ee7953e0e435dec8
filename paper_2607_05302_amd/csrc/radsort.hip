// Host side of the Radsort library: argument checks, workspace layout, the
// launch sequence of Alg. 2 on a HIP stream, and the C ABI of include/radsort.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/radsort.h"
#include "common.hpp"
#include "kernels_state.hpp"
#include "kernel_round.hpp"
#include "kernels_prefix.hpp"
#include "kernels_small.hpp"
#include "kernels_wg.hpp"
#include "kernels_finalize.hpp"
#include "kernels_finalize_seq.hpp"

using namespace rs;

namespace {

thread_local hipError_t g_last_hip = hipSuccess;
#ifdef RS_TIMELINE
uint64_t* g_tl = nullptr;  // stamps of the Radsort round kernel (timeline builds)
uint64_t g_tl_tiles = 0;
#endif
// statistics and phase events of the last sort call, per host thread
thread_local radsort_stats g_stats{};

#define RS_HIP(call)                                 \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) {                      \
            g_last_hip = e_;                         \
            return RADSORT_E_DEVICE;                 \
        }                                            \
    } while (0)

constexpr uint32_t kRingWords = 1u << 19;  // look-back ring: 2^ring_log2 * sigma count words
constexpr uint32_t kSuperSlotsLog2 = 16;   // slots per super-tile: 2^16 (8 tiles of 8192)

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

int ilog2(uint64_t x)
{
    int r = 0;
    while ((1ull << r) < x) r++;
    return r;
}

// Shape of the round kernel's workgroup per record size (KB key bytes, VB payload
// bytes), digit width (WIDE: more than 8 bits) and round (OOP: Alg. 1).  E = 64 *
// WAVES * ITEMS slots per tile.  The shape decides how many workgroups share a
// compute unit: the staged tile and per-wave digit counts must fit its 160 KB of
// LDS, the records held in registers its register file.
//   shape 0: one workgroup per CU, the next tile's records loaded into registers
//     while the current one is processed (PF), the payload staged beside the keys;
//   shape 1: two workgroups per CU (at most 128 VGPRs and about 68 KB of LDS
//     each): no register prefetch, the payload staged after the keys are written
//     out (SPLIT).  Measured at 2^28 uint32 + uint32, b = 2048: Radsort round
//     1.59 ms against 2.07 ms for shape 0, with one workgroup per tile;
//   shapes 2-4 (tiles of 4096 slots, two to three workgroups per CU) measured
//     slower (2.10-2.42 ms against 1.56 ms for shape 1, the same day), shapes
//     5-6 (16 waves of 8 slots) spill registers;
//     they are kept for measurement only (RS_ROUND_CFG selects a shape at build
//     time, RS_RADSORT_FORM the launch form of the Radsort round).
// The out-of-place round keeps shape 0 (1.50 ms, against 2.36 ms with shape 1).
#ifndef RS_ROUND_CFG
#define RS_ROUND_CFG 1
#endif
template <int KB, int VB, bool WIDE, bool OOP = false> struct TileCfg {
    static constexpr int C = (WIDE || OOP) ? 0 : RS_ROUND_CFG;
    static constexpr bool BIG = KB + VB >= 12;
    static constexpr bool NARROW = KB == 4 && VB <= 4;  // 8 bytes or less per record
    static constexpr int WAVES = WIDE ? 4 : (C == 3 ? 4 : C >= 5 ? 16 : 8);
    static constexpr int ITEMS = C == 0 ? (BIG ? 8 : 16)
                               : C == 1 ? (NARROW ? 16 : 8)
                               : C == 3 ? (BIG ? 8 : 16)
                               : C >= 5 ? 8
                                        : 8;
    static constexpr bool PF = C == 0 || C == 4;
    static constexpr bool SPLIT = C != 0;
    static constexpr int OCC = C == 0 ? 1 : C == 2 ? 6 : C == 5 ? 8 : C == 6 ? 6 : 4;
    using Shape = RoundShape<WAVES, ITEMS, PF, SPLIT, OCC>;
    static constexpr int E = 64 * WAVES * ITEMS;
};

// The Radsort round's tile for large arrays of records of at most 8 bytes: shape 1
// with twice the slots per lane (4-byte keys: 16384-slot tiles; 8-byte keys without
// payload: 8192), one workgroup per compute unit.  Its digit runs per tile are twice
// as long and the super-tiles half as many.  Measured with 8-bit digits: uint32 +
// uint32 at 2^28, b = 2048, 8.20-8.27 ms per sort against 8.47 ms with the smaller
// tile (from 2^25 to 2^27 elements no faster: fewer tiles in flight, so it is taken
// from kLargeTileMin on); uint64 keys at b = 4096, 18.8 against 19.6 ms at 2^28 and
// 76.5 against 81.1 ms at 2^30.
template <int KB> struct LargeTile {  // KB = 4: keys of 4 bytes; 8: keys of 8 bytes, no payload
    static constexpr int WAVES = 8, ITEMS = KB == 4 ? 32 : 16;
    using Shape = RoundShape<WAVES, ITEMS, false, true, 2>;
    static constexpr int E = 64 * WAVES * ITEMS;
};
constexpr uint64_t kLargeTileMin = 1ull << 28;  // elements

struct Geo {
    uint64_t n = 0;
    uint32_t kb = 0, vb = 0, bits = 0, sigma = 0, nt = 0, b = 0, log2b = 0;
    uint64_t nb = 0;
    uint32_t npi = 0, E = 0, tiles = 0, ring_w = 0, ring_log2 = 0;
    uint32_t st_log2 = 0;                 // tiles per super-tile: 2^st_log2
    uint32_t supers = 0, oop_supers = 0;  // super-tiles of a Radsort / out-of-place round
    uint32_t oop_E = 0, oop_st_log2 = 0;  // tile and super-tile of the out-of-place round
    bool fin_temps = false;       // finalize scratch holds the two-kernel F1's temporary blocks
    bool fin_temps_pack = false;  // the same for a packed state (n_pi + sigma blocks)
    bool pack_ok = false;         // one-call sorts pack the last round (plan_round)
    bool large_tile = false;      // the Radsort round runs LargeTile (E = 16384)
};

// Workspace regions (byte offsets), each 256-byte aligned.
struct Layout {
    uint64_t Tk, Tv, pi0, pi1, blen, opened, S, Pidx, Plen, f, est, ctr, ring, agg, done,
        csum, stcnt, fin, alt_k, alt_v;
    uint64_t Xk, Xv, pack;  // a packed last round only: sigma extra blocks, bucket table
    uint64_t consumed;  // ordering-check builds only: a tag per physical block
    uint64_t ring_bytes, fin_bytes, total;
};

template <bool WIDE, bool OOP> uint32_t tile_elems_t(uint32_t kb, uint32_t vb)
{
    if (kb == 4 && vb == 0) return TileCfg<4, 0, WIDE, OOP>::E;
    if (kb == 4 && vb == 4) return TileCfg<4, 4, WIDE, OOP>::E;
    if (kb == 4 && vb == 8) return TileCfg<4, 8, WIDE, OOP>::E;
    if (kb == 8 && vb == 0) return TileCfg<8, 0, WIDE, OOP>::E;
    if (kb == 8 && vb == 4) return TileCfg<8, 4, WIDE, OOP>::E;
    return TileCfg<8, 8, WIDE, OOP>::E;
}

// digits of more than 8 bits take the wide tile (per-wave counts of 2^11 digits)
uint32_t tile_elems(uint32_t kb, uint32_t vb, uint32_t bits, bool oop)
{
    if (bits > 8) return oop ? tile_elems_t<true, true>(kb, vb) : tile_elems_t<true, false>(kb, vb);
    return oop ? tile_elems_t<false, true>(kb, vb) : tile_elems_t<false, false>(kb, vb);
}

// Compute units of the current device; 256 (an MI355X) when no device answers.
uint32_t device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    return (uint32_t)cus;
}

int make_geo(Geo& g, uint64_t n, int key_bytes, int payload_bytes, int digit_bits,
             const radsort_opts* opts)
{
    if (key_bytes != 4 && key_bytes != 8) return RADSORT_E_INVALID;
    if (payload_bytes != 0 && payload_bytes != 4 && payload_bytes != 8) return RADSORT_E_INVALID;
    if (digit_bits < 1 || digit_bits > 16) return RADSORT_E_INVALID;
    // 12 .. 16 bits: 2 sigma b head-block elements, waves * sigma LDS counts and
    // digit runs shorter than a line per tile cost more than the round they save
    if (digit_bits > 11) return RADSORT_E_UNSUPPORTED;
#ifndef RS_DEBUG_ORDER
    if (opts && (opts->flags & RADSORT_F_DEBUG_ORDER)) return RADSORT_E_UNSUPPORTED;
#endif
    uint32_t b = (opts && opts->block_elems) ? opts->block_elems : 1024u;
    if (b < 64 || b > 65536 || (b & (b - 1))) return RADSORT_E_INVALID;
    if (n >= (1ull << 32)) return RADSORT_E_UNSUPPORTED;
    g.n = n;
    g.kb = key_bytes;
    g.vb = payload_bytes;
    g.bits = digit_bits;
    g.sigma = 1u << digit_bits;
    g.nt = (8 * key_bytes + digit_bits - 1) / digit_bits;
    g.b = b;
    g.log2b = ilog2(b);
    g.nb = n >> g.log2b;
    uint64_t npi = g.nb + 2ull * g.sigma;  // state table, Sec. 2.1
    // pi entries are 32-bit with the top bit free; finalize scans at most 4096^2 entries
    if (npi >= (uint64_t)kScanTile * kScanTile) return RADSORT_E_UNSUPPORTED;
    g.npi = (uint32_t)npi;
    g.large_tile = digit_bits <= 8 && n >= kLargeTileMin &&
                   ((key_bytes == 4 && payload_bytes <= 4) || (key_bytes == 8 && payload_bytes == 0));
    g.E = !g.large_tile ? tile_elems(g.kb, g.vb, g.bits, false)
          : key_bytes == 4 ? (uint32_t)LargeTile<4>::E : (uint32_t)LargeTile<8>::E;
    g.oop_E = tile_elems(g.kb, g.vb, g.bits, true);
#ifdef RS_DEBUG_ORDER
    if (opts && (opts->flags & RADSORT_F_DEBUG_ORDER) && g.b > g.E) return RADSORT_E_UNSUPPORTED;
#endif
    // input slots of a round: at most (floor(n/b) + sigma) blocks of b
    uint64_t slots = (g.nb + g.sigma) << g.log2b;
    g.tiles = (uint32_t)((slots + g.E - 1) / g.E);
    // ring slots (a power of two): one per tile when the tiles fit, else the cap;
    // with a slot per tile no slot is ever reused
    const uint32_t ring_cap = std::max<uint32_t>(256u, kRingWords / g.sigma);
    uint32_t ring_w = 32;
    while (ring_w < g.tiles && ring_w < ring_cap) ring_w <<= 1;
    g.ring_w = ring_w;
    g.ring_log2 = ilog2(g.ring_w);
    // a super-tile spans at least 2^kSuperSlotsLog2 slots and at least one block
    auto super_log2 = [&](uint32_t E) {
        const uint32_t elog = (uint32_t)ilog2(E);
        return std::max<uint32_t>(kSuperSlotsLog2 > elog ? kSuperSlotsLog2 - elog : 0u,
                                  g.log2b > elog ? g.log2b - elog : 0u);
    };
    g.st_log2 = super_log2(g.E);
    g.supers = (g.tiles + (1u << g.st_log2) - 1) >> g.st_log2;
    g.oop_st_log2 = super_log2(g.oop_E);
    const uint64_t oop_tiles = (n + g.oop_E - 1) / g.oop_E;
    g.oop_supers = (uint32_t)((oop_tiles + (1u << g.oop_st_log2) - 1) >> g.oop_st_log2);
    // F1 of finalize runs cooperatively on one workgroup per compute unit unless the
    // GPU is shared or that grid cannot cover the state; only the other form needs
    // temporary blocks in the workspace
    const bool shared = opts && (opts->flags & RADSORT_F_SHARED);
    const uint32_t cus = device_cus();
    g.fin_temps = shared || !fin_coop(g.npi, g.b, g.kb + g.vb, cus).covers;
    // the packed last round: its finalize is F1 over n_pi + sigma blocks, then the
    // spare blocks' slots copied into place (no compaction)
    g.fin_temps_pack = shared || !fin_coop(g.npi + g.sigma, g.b, g.kb + g.vb, cus).covers;
    g.pack_ok = true;
#ifdef RS_DEBUG_ORDER
    g.pack_ok = false;  // the ordering check follows the rounds of the paper
#endif
    return RADSORT_OK;
}

// Finalize scratch (parallel Alg. 7): see kernels_finalize.hpp.
uint64_t finalize_bytes(const Geo& g, bool pack)
{
    return fin_scratch_bytes(g.npi + (pack ? g.sigma : 0u), g.n, g.b, g.kb + g.vb,
                             pack ? g.fin_temps_pack : g.fin_temps);
}

// pack: the workspace of a sort whose last round is packed (Geo::pack_ok): sigma
// extra blocks, and the block permutations and finalize arrays over n_pi + sigma
// blocks.  The small arrays come first, so that the error word's place depends
// on n_t and sigma only.
Layout make_layout(const Geo& g, bool oop, bool pack = false)
{
    Layout L{};
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    const uint64_t sig = g.sigma, nt = g.nt;
    pack = pack && !oop;
    L.S = take(4 * nt * sig);
    L.Pidx = take(4 * (nt + 1) * sig);
    L.Plen = take(4 * (nt + 1) * sig);
    L.f = take(4 * (nt + 1));
    L.est = take(4 * nt * sig);
    L.ctr = take(4 * (nt + 8));
    if (!oop) {
        const uint64_t npx = g.npi + (pack ? sig : 0);
        L.Tk = take(2 * sig * g.b * g.kb);
        L.Tv = take(2 * sig * g.b * g.vb);
        L.pi0 = take(4ull * npx);
        L.pi1 = take(4ull * npx);
        L.blen = take(4ull * npx);
        L.opened = take(8ull * g.sigma);
        if (pack) {
            L.Xk = take(sig * g.b * g.kb);
            L.Xv = take(sig * g.b * g.vb);
            L.pack = take(4 * (2 * sig + 2));
        }
    } else {
        L.alt_k = take(g.n * g.kb);
        L.alt_v = take(g.n * g.vb);
    }
#ifdef RS_DEBUG_ORDER
    L.consumed = oop ? 0 : take(4ull * g.npi);
#endif
    // the look-back ring (count words, done words) and the chunk sums of the
    // super-tile scan, zeroed before each round; then the super-tile digit starts.
    // Finalize reuses all of it.
    const uint64_t supers = oop ? g.oop_supers : g.supers;
    const uint64_t agg_bytes = 4ull * g.ring_w * sig;
    // + the tile counter of the round kernel and the counter of the counting kernel
    const uint64_t done_bytes = align_up(4ull * g.ring_w + 8, 256);
    // one more row than super-tiles: the column scan leaves the digit totals there
    const uint64_t csum_bytes = align_up(4ull * ((supers + kScanRows) / kScanRows) * sig, 256);
    L.ring_bytes = agg_bytes + done_bytes + csum_bytes;
    const uint64_t st_bytes = align_up(4ull * (supers + 1) * sig, 256);
    L.fin_bytes = oop ? 0 : finalize_bytes(g, pack);
    L.ring = take(std::max(L.ring_bytes + st_bytes, L.fin_bytes));
    L.agg = L.ring;
    L.done = L.ring + agg_bytes;
    L.csum = L.done + done_bytes;
    L.stcnt = L.ring + L.ring_bytes;
    L.fin = L.ring;
    L.total = o;
    return L;
}

// HIP events recorded on the call's stream around each phase (RADSORT_F_TIMING).
enum Mark { kStart, kSetupEnd, kCountBegin, kRoundBegin, kRoundEnd, kFixupEnd, kFinBegin, kFinEnd };

struct Timer {
    static constexpr int kMax = 8 + 4 * RADSORT_MAX_ROUNDS;
    hipEvent_t ev[kMax];
    int tag[kMax], round[kMax];
    int count = 0;
    bool created = false, active = false, pending = false;

    void begin()
    {
        if (!created) {
            for (int i = 0; i < kMax; i++) (void)hipEventCreate(&ev[i]);
            created = true;
        }
        count = 0;
        active = true;
        pending = false;
    }
    void mark(Mark m, int r, hipStream_t s)
    {
        if (!active || count >= kMax) return;
        tag[count] = m;
        round[count] = r;
        (void)hipEventRecord(ev[count], s);
        count++;
    }
    void end()
    {
        if (active) pending = count > 0;
        active = false;
    }
    // waits for the last event and fills the timing fields of st
    void report(radsort_stats& st)
    {
        if (!pending) return;
        pending = false;
        if (hipEventSynchronize(ev[count - 1]) != hipSuccess) return;
        auto ms = [&](int a, int b) {
            float t = 0;
            (void)hipEventElapsedTime(&t, ev[a], ev[b]);
            return t;
        };
        st.timed = 1;
        st.setup_ms = st.fixup_ms = st.finalize_ms = 0;
        for (int r = 0; r < RADSORT_MAX_ROUNDS; r++) st.round_ms[r] = st.count_ms[r] = 0;
        st.total_ms = ms(0, count - 1);
        for (int i = 1; i < count; i++) {
            const float d = ms(i - 1, i);
            switch (tag[i]) {
            case kSetupEnd: st.setup_ms += d; break;
            case kRoundEnd: st.round_ms[round[i] % RADSORT_MAX_ROUNDS] += d; break;
            case kRoundBegin: st.count_ms[round[i] % RADSORT_MAX_ROUNDS] += d; break;
            case kCountBegin:
            case kFixupEnd: st.fixup_ms += d; break;
            case kFinEnd: st.finalize_ms += d; break;
            default: st.setup_ms += d; break;  // gaps before a finalize
            }
        }
    }
};

thread_local Timer g_timer;

void launch_fill(uint32_t* p, uint64_t count, uint32_t v, hipStream_t s)
{
    if (!count) return;
    uint32_t grid = (uint32_t)std::min<uint64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, count, v);
}

}  // namespace

struct radsort_state {
    Geo g;
    Layout L;
    uint8_t* ws = nullptr;
    bool own_ws = false;
    void* keys = nullptr;
    void* vals = nullptr;
    uint32_t rounds_done = 0;  // rounds since setup
    int cur = 0;               // which pi buffer holds pi
    uint64_t count = 0;        // elements in the dataset (fewer after truncate)
    bool truncated = false;
    bool is_setup = false;
    bool dynamic = false;      // launch forms that need no co-residency (shared GPU)
    bool shared = false;       // other work shares the GPU: no cooperative launch at all
    bool seq_draws = false;    // draws in the sequential pool order (RADSORT_F_SEQ_DRAWS)
    bool pack = false;         // the last round is packed (workspace laid out for it)
    int msd_shift = -1;        // >= 0: the rounds sort the digit at this shift (MSD split)
    bool debug_order = false;  // ordering-check builds: RADSORT_F_DEBUG_ORDER
    bool debug_plant = false;  // ... and RADSORT_F_DEBUG_PLANT: marks with a wrong tag
    uint32_t debug_seq = 0;    // the state's number, part of the round tags

    uint32_t* u32(uint64_t off) const { return (uint32_t*)(ws + off); }
    uint32_t* pi(int which) const { return u32(which ? L.pi1 : L.pi0); }
    PlanPtrs plan() const
    {
        return PlanPtrs{u32(L.S), u32(L.Pidx), u32(L.Plen), u32(L.f), u32(L.est)};
    }
    uint32_t* err() const { return u32(L.ctr) + g.nt; }
};

namespace {

// ---- launch helpers templated on key / payload widths --------------------------------

template <int KB> int launch_histograms(const void* keys, const Geo& g, uint32_t* hist,
                                        hipStream_t s)
{
    launch_fill(hist, (uint64_t)g.nt * g.sigma, 0, s);
    if (g.n == 0) return RADSORT_OK;
    // copies of the counts per workgroup: as many as fit in 32 KB, up to one per wave
    const uint32_t words = g.nt * g.sigma;
    const uint32_t copies = std::max<uint32_t>(1, std::min<uint32_t>(8, 8192 / words));
    uint32_t grid = (uint32_t)std::min<uint64_t>((g.n + 4095) / 4096, 2048);
    hipLaunchKernelGGL((k_histograms<KB, 512>), dim3(grid), dim3(512), 4 * copies * words, s,
                       (const typename UInt<KB>::T*)keys, g.n, g.bits, g.nt, copies, hist);
    return RADSORT_OK;
}

// Workgroups of `kern` that fit on the device at once (cached per device).
int resident_capacity(const void* kern, uint32_t threads)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, kern});
    if (it != cache.end()) return it->second;
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, (int)threads, 0) != hipSuccess)
        return 0;
    cache[{dev, kern}] = cus * per;
    return cus * per;
}

// The round kernel is persistent: at most as many workgroups as fit at once, all
// resident (cooperative launch), each taking tiles in grid-stride order.
template <typename Args>
int launch_persistent(const void* kern, uint32_t tiles, uint32_t threads, Args& a, hipStream_t s)
{
    const int cap = resident_capacity(kern, threads);
    if (cap <= 0) return RADSORT_E_DEVICE;
    const uint32_t grid = std::min<uint32_t>(tiles, (uint32_t)cap);
    static const bool verbose = getenv("RADSORT_VERBOSE") != nullptr;
    if (verbose)
        fprintf(stderr, "radsort: persistent launch %u workgroups x %u threads for %u tiles\n",
                grid, threads, tiles);
    void* args[] = {(void*)&a};
    RS_HIP(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(threads), args, 0, s));
    return RADSORT_OK;
}

// Digit counts of every super-tile of a round's input, then their column scan:
// stcnt[u][d] = elements with digit d before super-tile u, for u = 0 .. supers;
// row `supers` (past the input, counted as empty) ends with the digit totals of
// the round's input, from which the scan's last workgroup makes the plan of round
// r (S[r], P[r+1], f[r+1], and est[r] for the out-of-place round).
template <int KB, bool OOP>
void launch_super_counts(const Geo& g, const typename UInt<KB>::T* Ak,
                         const typename UInt<KB>::T* Tk, const uint32_t* pi,
                         const uint32_t* blen, const uint32_t* f_in, uint32_t shift,
                         uint32_t* stcnt, uint32_t* csum, uint32_t* err, uint32_t* done_ctr,
                         uint32_t r, PlanPtrs p, hipStream_t s, bool packed = false)
{
    const uint32_t rows = (OOP ? g.oop_supers : g.supers) + 1;
    const uint32_t sts_log2 = OOP ? g.oop_st_log2 + (uint32_t)ilog2(g.oop_E)
                                  : g.st_log2 + (uint32_t)ilog2(g.E);
    const uint32_t sig = g.sigma, plan = OOP ? 2u : packed ? 3u : 1u;
    PlanPtrs pr{p.S + r * sig, p.Pidx + (r + 1) * sig, p.Plen + (r + 1) * sig, p.f + r + 1,
                p.est + r * sig};
    // one chunk of rows: the counting kernel's last workgroup scans and plans
    const bool fused = rows <= kScanRows;
    hipLaunchKernelGGL((k_supertile_counts<KB, OOP, 1024>), dim3(rows), dim3(1024), 0, s, Ak, Tk,
                       pi, blen, f_in, g.n, shift, g.bits, g.log2b, g.npi, sts_log2, stcnt, csum,
                       err, done_ctr, fused ? plan : 0u, pr);
    if (!fused)
        hipLaunchKernelGGL(k_column_scan<256>, dim3((rows + kScanRows - 1) / kScanRows),
                           dim3(256), 4 * (2 * sig + 8), s, stcnt, csum, rows, sig, g.log2b, plan,
                           pr);
}

// The claimed forms (no co-residency needed): one workgroup per tile, or for the
// claim loop at most as many workgroups as fit at once.
template <typename Args>
int launch_dynamic(const void* kern, uint32_t tiles, uint32_t threads, Args& a, hipStream_t s,
                   bool loop)
{
    uint32_t grid = tiles;
    if (loop) {
        const int cap = resident_capacity(kern, threads);
        if (cap <= 0) return RADSORT_E_DEVICE;
        grid = std::min<uint32_t>(tiles, (uint32_t)cap);
    }
    void* args[] = {(void*)&a};
    RS_HIP(hipLaunchKernel(kern, dim3(grid), dim3(threads), args, 0, s));
    return RADSORT_OK;
}

#ifndef RS_RADSORT_FORM
#define RS_RADSORT_FORM kPerTile
#endif
// seq: draws in the sequential pool order (pi as in the sequential algorithm);
// otherwise in (digit, block) order within a tile.  Digits of more than 8 bits
// always draw in the sequential order.  The out-of-place round draws nothing.
template <int KB, int VB, bool OOP>
int launch_round_t(const Geo& g, TileArgs<KB, VB>& a, hipStream_t s, bool dyn = false,
                   bool seq = true)
{
    using N = TileCfg<KB, VB, false, OOP>;
    using Wd = TileCfg<KB, VB, true, OOP>;
    using NS = typename N::Shape;
    const uint32_t tiles = OOP ? (uint32_t)((g.n + g.oop_E - 1) / g.oop_E) : g.tiles;
    if (tiles == 0) return RADSORT_OK;
    if constexpr (!OOP && ((KB == 4 && VB <= 4) || (KB == 8 && VB == 0))) {
        if (g.large_tile) {  // 8-bit or narrower digits only (make_geo); a workgroup per tile
            using LS = typename LargeTile<KB>::Shape;
            constexpr int M = RS_RADSORT_FORM;
            const void* kern =
                seq ? (g.bits == 8 ? (const void*)&k_round<KB, VB, false, 8, 256, LS, M, true>
                                   : (const void*)&k_round<KB, VB, false, 0, 256, LS, M, true>)
                    : (g.bits == 8 ? (const void*)&k_round<KB, VB, false, 8, 256, LS, M, false>
                                   : (const void*)&k_round<KB, VB, false, 0, 256, LS, M, false>);
            return launch_dynamic(kern, tiles, 64 * LargeTile<KB>::WAVES, a, s, false);
        }
    }
    // shapes without register prefetch take a workgroup per tile (the persistent
    // form would hold the loop's state in registers the shape does not have)
    if (g.bits <= 8 && !N::PF) dyn = true;
    if (dyn) {
        // measured alone: one workgroup per tile for the Radsort round, the claim
        // loop for the out-of-place round
        constexpr int M = OOP ? kClaimLoop : RS_RADSORT_FORM;
        const uint32_t nt = 64 * N::WAVES;
        const void* kern;
        if (OOP || !seq)
            kern = g.bits == 8 ? (const void*)&k_round<KB, VB, OOP, 8, 256, NS, M, false>
                               : (const void*)&k_round<KB, VB, OOP, 0, 256, NS, M, false>;
        else
            kern = g.bits == 8 ? (const void*)&k_round<KB, VB, OOP, 8, 256, NS, M, true>
                               : (const void*)&k_round<KB, VB, OOP, 0, 256, NS, M, true>;
        if (g.bits <= 8) return launch_dynamic(kern, tiles, nt, a, s, OOP);
        return launch_dynamic(
            (const void*)&k_round<KB, VB, OOP, 0, 2048, typename Wd::Shape, M, !OOP>, tiles,
            64 * Wd::WAVES, a, s, OOP);
    }
    if constexpr (N::PF) {
        const void* kern;
        if (OOP || !seq)
            kern = g.bits == 8 ? (const void*)&k_round<KB, VB, OOP, 8, 256, NS, kPersistent, false>
                               : (const void*)&k_round<KB, VB, OOP, 0, 256, NS, kPersistent, false>;
        else
            kern = g.bits == 8 ? (const void*)&k_round<KB, VB, OOP, 8, 256, NS, kPersistent, true>
                               : (const void*)&k_round<KB, VB, OOP, 0, 256, NS, kPersistent, true>;
        if (g.bits <= 8) return launch_persistent(kern, tiles, 64 * N::WAVES, a, s);
    }
    return launch_persistent(
        (const void*)&k_round<KB, VB, OOP, 0, 2048, typename Wd::Shape, kPersistent, !OOP>, tiles,
        64 * Wd::WAVES, a, s);
}

template <int KB, int VB> struct Ops {
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;

    static int setup(radsort_state* st, hipStream_t s)
    {
        const Geo& g = st->g;
        g_timer.mark(kStart, 0, s);
        // every round is planned later from its own digit counts
        launch_fill(st->u32(st->L.ctr), g.nt + 8, 0, s);
        uint64_t work = std::max<uint64_t>(g.npi, g.n & (g.b - 1));
        uint32_t grid = (uint32_t)std::min<uint64_t>((work + 255) / 256, 4096);
        hipLaunchKernelGGL((k_setup<KB, VB>), dim3(grid), dim3(256), 0, s, (K*)st->keys,
                           (V*)st->vals, (K*)(st->ws + st->L.Tk), (V*)(st->ws + st->L.Tv), g.n,
                           g.log2b, g.sigma, g.npi, st->pi(0), st->pi(1), st->u32(st->L.blen),
                           (uint64_t*)(st->ws + st->L.opened), st->u32(st->L.Pidx),
                           st->u32(st->L.Plen), st->u32(st->L.f), st->u32(st->L.ring),
                           st->L.ring_bytes / 4);
        g_timer.mark(kSetupEnd, 0, s);
        st->cur = 0;
        st->rounds_done = 0;
        st->count = g.n;
        st->truncated = false;
        st->is_setup = true;
        return RADSORT_OK;
    }

    // truncate (Alg. 8) between rounds; the rounds still to run plan themselves
    // from the shorter dataset
    static int truncate(radsort_state* st, uint64_t count, hipStream_t s)
    {
        const Geo& g = st->g;
        const uint32_t r = st->rounds_done;
        hipLaunchKernelGGL(k_truncate<256>, dim3(1), dim3(256), 4 * g.sigma, s,
                           st->u32(st->L.Pidx) + r * g.sigma, st->u32(st->L.Plen) + r * g.sigma,
                           st->u32(st->L.f) + r, st->u32(st->L.blen), g.sigma, g.log2b, count,
                           st->err());
        st->count = count;
        st->truncated = true;
        return RADSORT_OK;
    }

    // a new sort of the current contents: the state becomes the input of round 0
    static int restart(radsort_state* st, hipStream_t s)
    {
        const Geo& g = st->g;
        const uint32_t r = st->rounds_done;
        if (r) {
            hipLaunchKernelGGL(k_copy_u32, dim3((g.sigma + 255) / 256), dim3(256), 0, s,
                               st->u32(st->L.Pidx), st->u32(st->L.Pidx) + r * g.sigma, g.sigma);
            hipLaunchKernelGGL(k_copy_u32, dim3((g.sigma + 255) / 256), dim3(256), 0, s,
                               st->u32(st->L.Plen), st->u32(st->L.Plen) + r * g.sigma, g.sigma);
            hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, s, st->u32(st->L.f),
                               st->u32(st->L.f) + r, 1u);
        }
        st->rounds_done = 0;
        return RADSORT_OK;
    }

    static int blocks(radsort_state* st, uint32_t* phys, uint32_t* len, hipStream_t s)
    {
        const Geo& g = st->g;
        const uint32_t m = g.npi - g.sigma;
        const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((m + 255) / 256, 4096));
        hipLaunchKernelGGL(k_block_table, dim3(grid), dim3(256), 0, s, st->pi(st->cur),
                           st->u32(st->L.blen), st->u32(st->L.f) + st->rounds_done, g.sigma,
                           g.npi, g.log2b, phys, len);
        return RADSORT_OK;
    }

    static int round(radsort_state* st, hipStream_t s)
    {
        const Geo& g = st->g;
        const uint32_t r = st->rounds_done;
        const uint32_t t = g.nt - 1 - r;  // key position of this round
        TileArgs<KB, VB> a{};
        (void)t;
        a.Ak = (K*)st->keys;
        a.Av = (V*)st->vals;
        a.Tk = (K*)(st->ws + st->L.Tk);
        a.Tv = (V*)(st->ws + st->L.Tv);
        a.pi_old = st->pi(st->cur);
        a.pi_new = st->pi(st->cur ^ 1);
        a.blen = st->u32(st->L.blen);
        a.f_in = st->u32(st->L.f) + r;
        a.S = st->u32(st->L.S) + r * g.sigma;
        a.opened = (uint64_t*)(st->ws + st->L.opened);
        a.agg = (uint32_t*)(st->ws + st->L.agg);
        a.done = (uint32_t*)(st->ws + st->L.done);
        a.err = st->err();
        a.tile_ctr = a.done + g.ring_w;  // zeroed with the ring
        a.shift = st->msd_shift >= 0 ? (uint32_t)st->msd_shift : g.bits * r;
        a.bits = g.bits;
        a.log2b = g.log2b;
        a.npi = g.npi;
        a.ring_log2 = g.ring_log2;
        a.st_log2 = g.st_log2;
        // the last round of a packed sort (plan_round, k_round): its buckets start at
        // their final offsets and it draws from sigma extra blocks first
        const bool packed = st->pack && r + 1 == g.nt && st->msd_shift < 0;
        a.npi_x = packed ? g.npi + g.sigma : g.npi;
        if (packed) {
            a.pack_est = st->u32(st->L.est) + r * g.sigma;
            a.Xk = (K*)(st->ws + st->L.Xk);
            a.Xv = (V*)(st->ws + st->L.Xv);
            launch_fill(a.pi_new + g.npi, g.sigma, kEmpty, s);  // entries past n_pi unset
        }
#ifdef RS_TIMELINE
        a.tl = g.tiles <= g_tl_tiles ? g_tl : nullptr;
#endif
#ifdef RS_DEBUG_ORDER
        a.consumed = st->debug_order ? st->u32(st->L.consumed) : nullptr;
        a.tag = st->debug_seq << 8 | (r + 1);  // one per state and round
        a.tag_mark = st->debug_plant ? a.tag ^ 0x80u : a.tag;
#endif
        uint32_t* stcnt = (uint32_t*)(st->ws + st->L.stcnt);
        a.stbase = stcnt;
        // the ring is clear: setup or the previous round's fixup cleared it
        g_timer.mark(kCountBegin, r, s);
        launch_super_counts<KB, false>(g, a.Ak, a.Tk, a.pi_old, a.blen, a.f_in, a.shift, stcnt,
                                       st->u32(st->L.csum), a.err, a.tile_ctr + 1, r,
                                       st->plan(), s, packed);
        g_timer.mark(kRoundBegin, r, s);
        int rc = launch_round_t<KB, VB, false>(g, a, s, st->dynamic, st->seq_draws);
        if (rc) return rc;
        g_timer.mark(kRoundEnd, r, s);
        uint32_t grid = (uint32_t)std::min<uint64_t>((a.npi_x + 255) / 256, 4096);
        if (packed)
            hipLaunchKernelGGL(k_pack_fixup, dim3(grid), dim3(256), 0, s, st->pi(st->cur),
                               st->pi(st->cur ^ 1), a.S, st->u32(st->L.f) + r + 1, g.sigma,
                               g.npi);
        else
            hipLaunchKernelGGL(k_fixup, dim3(grid), dim3(256), 0, s, st->pi(st->cur),
                               st->pi(st->cur ^ 1), a.S, st->u32(st->L.f) + r + 1,
                               st->u32(st->L.Pidx) + (r + 1) * g.sigma,
                               st->u32(st->L.Plen) + (r + 1) * g.sigma, st->u32(st->L.blen),
                               a.opened, g.sigma, g.log2b, g.npi, st->u32(st->L.ring),
                               st->L.ring_bytes / 4);
        g_timer.mark(kFixupEnd, r, s);
        st->cur ^= 1;
        st->rounds_done++;
        return RADSORT_OK;
    }

    static int finalize_seq(radsort_state* st, hipStream_t s)
    {
        const Geo& g = st->g;
        const uint32_t r = st->rounds_done;
        hipLaunchKernelGGL((k_finalize_seq<KB, VB, 1024>), dim3(1), dim3(1024), 0, s,
                           (K*)st->keys, (V*)st->vals, (K*)(st->ws + st->L.Tk),
                           (V*)(st->ws + st->L.Tv), st->pi(st->cur), st->u32(st->L.fin),
                           st->u32(st->L.Pidx) + r * g.sigma, st->u32(st->L.Plen) + r * g.sigma,
                           st->u32(st->L.f) + r, g.n, g.sigma, g.log2b, g.npi);
        return RADSORT_OK;
    }

    static int finalize(radsort_state* st, hipStream_t s)
    {
        const Geo& g = st->g;
        const uint32_t r = st->rounds_done;
        FinArgs<KB, VB> a{};
        a.Ak = (K*)st->keys;
        a.Av = (V*)st->vals;
        a.Tk = (K*)(st->ws + st->L.Tk);
        a.Tv = (V*)(st->ws + st->L.Tv);
        a.pi = st->pi(st->cur);
        a.Pidx = st->u32(st->L.Pidx) + r * g.sigma;
        a.Plen = st->u32(st->L.Plen) + r * g.sigma;
        a.f = st->u32(st->L.f) + r;
        a.n = g.n;
        a.sigma = g.sigma;
        a.log2b = g.log2b;
        a.npi = g.npi;
        a.npi_eq = g.npi;
        if (st->pack && r == g.nt && st->msd_shift < 0) {  // the last round was packed
            a.npi = g.npi + g.sigma;
            a.Xk = (K*)(st->ws + st->L.Xk);
            a.Xv = (V*)(st->ws + st->L.Xv);
            a.est = st->u32(st->L.est) + (r - 1) * g.sigma;
            a.S = st->u32(st->L.S) + (r - 1) * g.sigma;
            a.pack = st->u32(st->L.pack);
        }
        a.job = fin_job(a.npi);
        a.err = st->err();
        a.scratch = st->ws + st->L.fin;
        a.spare_pi = st->pi(st->cur ^ 1);
        a.spare_blen = st->u32(st->L.blen);
        g_timer.mark(kFinBegin, 0, s);
        int cap = 0;       // 0: the dynamic compaction
        uint32_t cus = 0;  // 0: F1 without a cooperative launch
        if (!st->dynamic) {
            const void* compact =
                (const void*)&k_fin_compact<KB, VB, fin_chunk<KB, VB>(), kCompactThreads>;
            cap = resident_capacity(compact, kCompactThreads);
            if (cap <= 0) return RADSORT_E_DEVICE;
        }
        if (!st->shared) {
            int dev = 0, n_cu = 0;
            RS_HIP(hipGetDevice(&dev));
            RS_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
            cus = (uint32_t)n_cu;
        }
        const bool temps = a.pack ? g.fin_temps_pack : g.fin_temps;
        const int fr = finalize_parallel<KB, VB>(a, (uint32_t)cap, cus, temps, s);
        int rc = fr == -2 ? RADSORT_E_NOMEM : fr ? RADSORT_E_DEVICE : RADSORT_OK;
        g_timer.mark(kFinEnd, 0, s);
        return rc;
    }

    static int logical(radsort_state* st, void* ok, void* ov, hipStream_t s)
    {
        const Geo& g = st->g;
        const uint32_t r = st->rounds_done;
        const uint32_t grid = g.npi - g.sigma;
        hipLaunchKernelGGL((k_gather_logical<KB, VB, 256>), dim3(grid), dim3(256), 0, s,
                           (const K*)st->keys, (const V*)st->vals,
                           (const K*)(st->ws + st->L.Tk), (const V*)(st->ws + st->L.Tv),
                           st->pi(st->cur), st->u32(st->L.Pidx) + r * g.sigma,
                           st->u32(st->L.Plen) + r * g.sigma, st->u32(st->L.f) + r, g.sigma,
                           g.log2b, g.npi, (K*)ok, (V*)ov);
        return RADSORT_OK;
    }

    // Alg. 1 rounds, ping-ponging between the caller's arrays and the workspace
    static int oop_sort(void* keys, void* vals, const Geo& g, const Layout& L, uint8_t* ws,
                        bool dyn, hipStream_t s)
    {
        // each round's element starts come from its own digit counts
        PlanPtrs p{(uint32_t*)(ws + L.S), (uint32_t*)(ws + L.Pidx), (uint32_t*)(ws + L.Plen),
                   (uint32_t*)(ws + L.f), (uint32_t*)(ws + L.est)};
        g_timer.mark(kStart, 0, s);
        uint32_t* ctr = (uint32_t*)(ws + L.ctr);
        launch_fill(ctr, g.nt + 8, 0, s);
        g_timer.mark(kSetupEnd, 0, s);
        K* bk[2] = {(K*)keys, (K*)(ws + L.alt_k)};
        V* bv[2] = {(V*)vals, (V*)(ws + L.alt_v)};
        for (uint32_t r = 0; r < g.nt; r++) {
            const uint32_t t = g.nt - 1 - r, from = r & 1;
            TileArgs<KB, VB> a{};
            a.Ak = bk[from];
            a.Av = bv[from];
            a.Tk = bk[from ^ 1];
            a.Tv = bv[from ^ 1];
            a.est = p.est + r * g.sigma;
            a.n = g.n;
            a.agg = (uint32_t*)(ws + L.agg);
            a.done = (uint32_t*)(ws + L.done);
            a.err = ctr + g.nt;
            a.tile_ctr = a.done + g.ring_w;  // zeroed with the ring
            a.shift = g.bits * (g.nt - 1 - t);
            a.bits = g.bits;
            a.log2b = g.log2b;
            a.ring_log2 = g.ring_log2;
            a.st_log2 = g.oop_st_log2;
            uint32_t* stcnt = (uint32_t*)(ws + L.stcnt);
            a.stbase = stcnt;
            launch_fill((uint32_t*)a.agg, L.ring_bytes / 4, 0, s);
            g_timer.mark(kCountBegin, r, s);
            launch_super_counts<KB, true>(g, a.Ak, (const K*)nullptr, nullptr, nullptr, nullptr,
                                          a.shift, stcnt, (uint32_t*)(ws + L.csum), a.err,
                                          a.tile_ctr + 1, r, p, s);
            g_timer.mark(kRoundBegin, r, s);
            int rc = launch_round_t<KB, VB, true>(g, a, s, dyn);
            if (rc) return rc;
            g_timer.mark(kRoundEnd, r, s);
        }
        g_timer.mark(kFinBegin, 0, s);
        if (g.nt & 1) {  // the result is in the workspace buffer: copy it back
            RS_HIP(hipMemcpyAsync(keys, bk[1], g.n * KB, hipMemcpyDeviceToDevice, s));
            if (VB) RS_HIP(hipMemcpyAsync(vals, bv[1], g.n * VB, hipMemcpyDeviceToDevice, s));
        }
        g_timer.mark(kFinEnd, 0, s);
        return RADSORT_OK;
    }
};

template <template <int, int> class F, typename... Args>
int dispatch(uint32_t kb, uint32_t vb, Args&&... args)
{
    if (kb == 4 && vb == 0) return F<4, 0>::run(args...);
    if (kb == 4 && vb == 4) return F<4, 4>::run(args...);
    if (kb == 4 && vb == 8) return F<4, 8>::run(args...);
    if (kb == 8 && vb == 0) return F<8, 0>::run(args...);
    if (kb == 8 && vb == 4) return F<8, 4>::run(args...);
    if (kb == 8 && vb == 8) return F<8, 8>::run(args...);
    return RADSORT_E_INVALID;
}

template <int KB, int VB> struct DoSetup {
    static int run(radsort_state* st, hipStream_t s) { return Ops<KB, VB>::setup(st, s); }
};
template <int KB, int VB> struct DoRound {
    static int run(radsort_state* st, hipStream_t s) { return Ops<KB, VB>::round(st, s); }
};
template <int KB, int VB> struct DoFinalize {
    static int run(radsort_state* st, hipStream_t s) { return Ops<KB, VB>::finalize(st, s); }
};
template <int KB, int VB> struct DoFinalizeSeq {
    static int run(radsort_state* st, hipStream_t s) { return Ops<KB, VB>::finalize_seq(st, s); }
};
template <int KB, int VB> struct DoTruncate {
    static int run(radsort_state* st, uint64_t count, hipStream_t s)
    {
        return Ops<KB, VB>::truncate(st, count, s);
    }
};
template <int KB, int VB> struct DoRestart {
    static int run(radsort_state* st, hipStream_t s) { return Ops<KB, VB>::restart(st, s); }
};
template <int KB, int VB> struct DoBlocks {
    static int run(radsort_state* st, uint32_t* phys, uint32_t* len, hipStream_t s)
    {
        return Ops<KB, VB>::blocks(st, phys, len, s);
    }
};
template <int KB, int VB> struct DoLogical {
    static int run(radsort_state* st, void* k, void* v, hipStream_t s)
    {
        return Ops<KB, VB>::logical(st, k, v, s);
    }
};
template <int KB, int VB> struct DoOop {
    static int run(void* k, void* v, const Geo& g, const Layout& L, uint8_t* ws, bool dyn,
                   hipStream_t s)
    {
        return Ops<KB, VB>::oop_sort(k, v, g, L, ws, dyn, s);
    }
};

int check_args(void* keys, void* payload, uint64_t n, int payload_bytes)
{
    if (n > 0 && !keys) return RADSORT_E_INVALID;
    if (payload_bytes && n > 0 && !payload) return RADSORT_E_INVALID;
    if (!payload_bytes && payload) return RADSORT_E_INVALID;
    return RADSORT_OK;
}

int read_err(radsort_state* st, hipStream_t s, uint32_t* bits)
{
    uint32_t e = 0;
    RS_HIP(hipMemcpyAsync(&e, st->err(), 4, hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    if (bits) *bits = e;
    g_stats.error_bits = e;
    return (e & kErrOrder) ? RADSORT_E_ORDER : e ? RADSORT_E_TIMEOUT : RADSORT_OK;
}

}  // namespace

// ---- C ABI ---------------------------------------------------------------------------


// ---- many arrays at once ---------------------------------------------------------

// Arrays of at most kSmallE<KB, VB> elements are sorted whole in LDS by
// k_sort_small (one workgroup each, no workspace).  Arrays up to wg_max_elems()
// are sorted by k_radsort_wg, one workgroup per array, all of them in one
// launch, each workgroup with its own T.  Larger ones run the Radsort steps in
// the dynamic launch form, spread over kSegLanes streams forked from the caller's
// stream, each lane with its own workspace.
constexpr uint32_t kSegLanes = 4;
template <int KB, int VB> struct SmallCfg {
    static constexpr int WAVES = 8;
    static constexpr int ITEMS = (KB + VB >= 12) ? 8 : 16;
    static constexpr uint32_t E = 64 * WAVES * ITEMS;
};
uint32_t small_elems(uint32_t kb, uint32_t vb) { return (kb + vb >= 12) ? 4096u : 8192u; }

struct SegChoice {
    uint32_t b, bits;
};

// block size and digit width for an array of n elements: the first class of the
// table whose max_log2n covers ceil(log2 n), else b = 2^ceil(log2 sqrt n) in
// [64, 2048] and 8-bit digits (b in Theta(sqrt n), Sec. 3)
SegChoice seg_choice(const radsort_seg_tuning* t, uint64_t n)
{
    const uint32_t lg = (uint32_t)ilog2(n);
    if (t)
        for (uint32_t c = 0; c < t->classes && c < RADSORT_SEG_CLASSES; c++)
            if (lg <= t->max_log2n[c] && t->block_elems[c]) return {t->block_elems[c], t->digit_bits[c]};
    const uint32_t b = std::min<uint32_t>(2048u, std::max<uint32_t>(64u, 1u << ((lg + 1) / 2)));
    return {b, 8u};
}

// The largest array the one-workgroup path takes: its limit, or lower when the
// tuning's first class with block_elems > 0 starts below it (arrays from that class
// on run on the lanes).  The host plan and the device list both use this bound.
uint64_t seg_wg_hi(const radsort_seg_tuning* t, uint64_t se)
{
    uint64_t hi = wg_max_elems();
    if (!t) return hi;
    for (uint32_t c = 0; c < t->classes && c < RADSORT_SEG_CLASSES; c++) {
        if (t->block_elems[c]) {
            const uint64_t below = c ? (1ull << std::min<uint32_t>(t->max_log2n[c - 1], 40)) : se;
            return std::max<uint64_t>(se, std::min<uint64_t>(hi, below));
        }
    }
    return hi;
}

struct SegPlan {
    std::vector<uint32_t> large;  // indices of the arrays that run the Radsort steps
    std::vector<uint32_t> lane;   // lane of each of them
    std::vector<SegChoice> choice;
    uint64_t wg_hi = 0;           // arrays of (small, wg_hi] elements take the one-workgroup path
    uint64_t lane_off[kSegLanes] = {}, lane_bytes[kSegLanes] = {};
    uint32_t wg_count = 0, wg_slots = 0;  // arrays of the one-workgroup path, workgroups
    uint64_t wg_off = 0, wg_slot_bytes = 0, wg_list_off = 0;
    uint64_t total = 0;
    bool any_small = false;
};

// Workgroups of the one-workgroup path (each with its own T); they never wait
// for each other, so they need not all be resident.
constexpr uint32_t kWgSlots = 256;

int make_seg_plan(SegPlan& P, const uint64_t* off, uint32_t nseg, int kb, int vb,
                  const radsort_seg_tuning* tuning, const radsort_opts* opts)
{
    const uint32_t se = small_elems(kb, vb);
    P.wg_hi = seg_wg_hi(tuning, se);
    std::vector<std::pair<uint64_t, uint32_t>> big;
    for (uint32_t i = 0; i < nseg; i++) {
        if (off[i + 1] < off[i]) return RADSORT_E_INVALID;
        const uint64_t n = off[i + 1] - off[i];
        if (n <= 1) continue;
        if (n <= se) {
            P.any_small = true;
            continue;
        }
        if (n <= P.wg_hi) {
            P.wg_count++;
            continue;
        }
        big.push_back({n, i});
    }
    // largest first, each to the lane with the fewest elements so far
    std::sort(big.begin(), big.end(), [](auto& x, auto& y) { return x.first > y.first; });
    uint64_t load[kSegLanes] = {};
    for (auto& [n, i] : big) {
        uint32_t l = 0;
        for (uint32_t k = 1; k < kSegLanes; k++)
            if (load[k] < load[l]) l = k;
        load[l] += n;
        SegChoice c = seg_choice(tuning, n);
        radsort_opts o = opts ? *opts : radsort_opts{};
        o.block_elems = c.b;
        o.flags |= RADSORT_F_SHARED;  // the lanes run concurrently (run_one)
        Geo g;
        int rc = make_geo(g, n, kb, vb, (int)c.bits, &o);
        if (rc) return rc;
        P.lane_bytes[l] = std::max(P.lane_bytes[l], make_layout(g, false, g.pack_ok).total);
        P.large.push_back(i);
        P.lane.push_back(l);
        P.choice.push_back(c);
    }
    uint64_t o = 256;  // error words and the one-workgroup path's claim counter
    for (uint32_t l = 0; l < kSegLanes; l++) {
        P.lane_off[l] = o;
        o = align_up(o + P.lane_bytes[l], 256);
    }
    if (P.wg_count) {
        P.wg_slots = std::min(P.wg_count, kWgSlots);
        P.wg_slot_bytes = wg_slot_bytes(kb, vb);
        P.wg_list_off = o;
        o = align_up(o + 4ull * P.wg_count, 256);
        P.wg_off = o;
        o += (uint64_t)P.wg_slots * P.wg_slot_bytes;
    }
    P.total = o;
    return RADSORT_OK;
}

struct LaneStreams {
    hipStream_t s[kSegLanes];
    hipEvent_t fork, join[kSegLanes];
};

// streams and events of the lanes, one set per device, kept until the process ends
int lane_streams(LaneStreams** out)
{
    static std::mutex mu;
    static std::map<int, LaneStreams*> sets;
    int dev = 0;
    RS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = sets.find(dev);
    if (it != sets.end()) {
        *out = it->second;
        return RADSORT_OK;
    }
    LaneStreams* L = new (std::nothrow) LaneStreams();
    if (!L) return RADSORT_E_NOMEM;
    for (uint32_t l = 0; l < kSegLanes; l++) {
        RS_HIP(hipStreamCreateWithFlags(&L->s[l], hipStreamNonBlocking));
        RS_HIP(hipEventCreateWithFlags(&L->join[l], hipEventDisableTiming));
    }
    RS_HIP(hipEventCreateWithFlags(&L->fork, hipEventDisableTiming));
    sets[dev] = L;
    *out = L;
    return RADSORT_OK;
}

template <int KB, int VB> struct DoSmall {
    static int run(void* keys, void* vals, const uint64_t* offsets_dev, uint32_t nseg,
                   uint32_t* err, hipStream_t s)
    {
        using C = SmallCfg<KB, VB>;
        const uint32_t nt = (8 * KB + 7) / 8;
        hipLaunchKernelGGL((k_sort_small<KB, VB, C::WAVES, C::ITEMS>), dim3(nseg),
                           dim3(64 * C::WAVES), 0, s, (typename UInt<KB>::T*)keys,
                           (typename Payload<VB>::T*)vals, offsets_dev, nseg, 8u, nt, err);
        return RADSORT_OK;
    }
};

template <int KB, int VB> struct DoWg {
    static int run(void* keys, void* vals, const uint64_t* offsets_dev, uint32_t nseg,
                   const SegPlan& P, uint8_t* ws, uint32_t* claim, uint32_t* err, hipStream_t s)
    {
        using C = WgCfg<KB, VB>;
        uint32_t* list = (uint32_t*)(ws + P.wg_list_off);
        hipLaunchKernelGGL(k_wg_list, dim3(1), dim3(1024), 0, s, offsets_dev, nseg,
                           (uint64_t)small_elems(KB, VB), P.wg_hi, list, P.wg_count);
        hipLaunchKernelGGL((k_radsort_wg<KB, VB>), dim3(P.wg_slots), dim3(C::NT), 0, s,
                           (typename UInt<KB>::T*)keys, (typename Payload<VB>::T*)vals,
                           offsets_dev, nseg, (const uint32_t*)list, P.wg_count, claim,
                           ws + P.wg_off, P.wg_slot_bytes, err);
        return RADSORT_OK;
    }
};

__global__ void k_or_error(const uint32_t* src, uint32_t* dst)
{
    if (threadIdx.x == 0 && *src) atomicOr(dst, *src);
}

// pack: the state's last round is packed (one-call sorts), its workspace laid out
// for that (make_layout)
static int state_create(radsort_state** out, void* keys, void* payload, uint64_t n, int key_bytes,
                 int payload_bytes, int digit_bits, const radsort_opts* opts, bool pack);

// the Radsort steps of one array on stream s, in the dynamic launch form; its
// device error bits are ORed into *errs
int run_one(void* keys, void* vals, uint64_t n, int kb, int vb, SegChoice c, uint8_t* ws,
            uint64_t ws_bytes, uint32_t* errs, hipStream_t s)
{
    radsort_opts o{};
    o.block_elems = c.b;
    o.flags = RADSORT_F_SHARED;  // sized as the plan sized it
    o.workspace = ws;
    o.workspace_bytes = ws_bytes;
    radsort_state* st = nullptr;
    int rc = state_create(&st, keys, vals, n, kb, vb, (int)c.bits, &o, true);
    if (rc) return rc;
    st->dynamic = true;
    st->shared = true;  // the lanes run concurrently: no cooperative launch
    rc = radsort_state_setup(st, s);
    for (uint32_t r = 0; !rc && r < st->g.nt; r++) rc = radsort_state_round(st, s);
    if (!rc) rc = radsort_state_finalize(st, s);
    if (!rc) hipLaunchKernelGGL(k_or_error, dim3(1), dim3(64), 0, s, st->err(), errs);
    radsort_state_destroy(st);
    return rc;
}

static int state_create(radsort_state** out, void* keys, void* payload, uint64_t n, int key_bytes,
                 int payload_bytes, int digit_bits, const radsort_opts* opts, bool pack)
{
    if (!out) return RADSORT_E_INVALID;
    *out = nullptr;
    int rc = check_args(keys, payload, n, payload_bytes);
    if (rc) return rc;
    Geo g;
    rc = make_geo(g, n, key_bytes, payload_bytes, digit_bits, opts);
    if (rc) return rc;
    radsort_state* st = new (std::nothrow) radsort_state();
    if (!st) return RADSORT_E_NOMEM;
    st->g = g;
    st->pack = pack && g.pack_ok;
    st->L = make_layout(g, false, st->pack);
    st->keys = keys;
    st->vals = payload;
    st->count = n;
    st->seq_draws = opts && (opts->flags & RADSORT_F_SEQ_DRAWS);
#ifdef RS_DEBUG_ORDER
    static std::atomic<uint32_t> debug_states{0};
    st->debug_order = opts && (opts->flags & RADSORT_F_DEBUG_ORDER);
    st->debug_plant = st->debug_order && (opts->flags & RADSORT_F_DEBUG_PLANT);
    st->debug_seq = (debug_states.fetch_add(1) + 1) & 0xFFFFFFu;
#endif
    if (opts && opts->workspace) {
        if (opts->workspace_bytes < st->L.total) {
            delete st;
            return RADSORT_E_NOMEM;
        }
        st->ws = (uint8_t*)opts->workspace;
    } else {
        hipError_t e = hipMalloc((void**)&st->ws, st->L.total);
        if (e != hipSuccess) {
            g_last_hip = e;
            delete st;
            return RADSORT_E_NOMEM;
        }
        st->own_ws = true;
    }
    *out = st;
    return RADSORT_OK;
}

extern "C" {

int radsort_state_create(radsort_state** out, void* keys, void* payload, uint64_t n,
                         int key_bytes, int payload_bytes, int digit_bits,
                         const radsort_opts* opts)
{
    return state_create(out, keys, payload, n, key_bytes, payload_bytes, digit_bits, opts, false);
}

int radsort_state_setup(radsort_state* st, void* stream)
{
    if (!st) return RADSORT_E_INVALID;
    int rc = dispatch<DoSetup>(st->g.kb, st->g.vb, st, (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

int radsort_state_round(radsort_state* st, void* stream)
{
    if (!st || !st->is_setup || st->rounds_done >= st->g.nt) return RADSORT_E_INVALID;
    int rc = dispatch<DoRound>(st->g.kb, st->g.vb, st, (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

int radsort_state_finalize(radsort_state* st, void* stream)
{
    if (!st || !st->is_setup) return RADSORT_E_INVALID;
    int rc = dispatch<DoFinalize>(st->g.kb, st->g.vb, st, (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    st->is_setup = false;
    return RADSORT_OK;
}

int radsort_state_finalize_sequential(radsort_state* st, void* stream)
{
    if (!st || !st->is_setup) return RADSORT_E_INVALID;
    if (st->truncated) return RADSORT_E_UNSUPPORTED;
    int rc = dispatch<DoFinalizeSeq>(st->g.kb, st->g.vb, st, (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    st->is_setup = false;
    return RADSORT_OK;
}

int radsort_state_read(radsort_state* st, uint32_t* pi, uint32_t* P_idx, uint32_t* P_len,
                       uint32_t* f, void* stream)
{
    if (!st) return RADSORT_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const Geo& g = st->g;
    const uint32_t r = st->rounds_done;
    if (pi) RS_HIP(hipMemcpyAsync(pi, st->pi(st->cur), 4ull * g.npi, hipMemcpyDeviceToHost, s));
    if (P_idx)
        RS_HIP(hipMemcpyAsync(P_idx, st->u32(st->L.Pidx) + r * g.sigma, 4ull * g.sigma,
                              hipMemcpyDeviceToHost, s));
    if (P_len)
        RS_HIP(hipMemcpyAsync(P_len, st->u32(st->L.Plen) + r * g.sigma, 4ull * g.sigma,
                              hipMemcpyDeviceToHost, s));
    if (f) RS_HIP(hipMemcpyAsync(f, st->u32(st->L.f) + r, 4, hipMemcpyDeviceToHost, s));
    return read_err(st, s, nullptr);
}

int radsort_state_truncate(radsort_state* st, uint64_t count, void* stream)
{
    if (!st || !st->is_setup || count > st->count) return RADSORT_E_INVALID;
    int rc = dispatch<DoTruncate>(st->g.kb, st->g.vb, st, count, (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

int radsort_state_restart(radsort_state* st, void* stream)
{
    if (!st || !st->is_setup) return RADSORT_E_INVALID;
    int rc = dispatch<DoRestart>(st->g.kb, st->g.vb, st, (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

int radsort_state_blocks(radsort_state* st, uint32_t* phys, uint32_t* len, void* stream)
{
    if (!st || !st->is_setup || (!phys && !len)) return RADSORT_E_INVALID;
    int rc = dispatch<DoBlocks>(st->g.kb, st->g.vb, st, phys, len, (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

int radsort_state_planes(const radsort_state* st, void** t_keys, void** t_payload,
                         uint32_t* block_elems)
{
    if (!st) return RADSORT_E_INVALID;
    if (t_keys) *t_keys = st->ws + st->L.Tk;
    if (t_payload) *t_payload = st->g.vb ? (void*)(st->ws + st->L.Tv) : nullptr;
    if (block_elems) *block_elems = st->g.b;
    return RADSORT_OK;
}

int radsort_state_count(const radsort_state* st, uint64_t* count)
{
    if (!st || !count) return RADSORT_E_INVALID;
    *count = st->count;
    return RADSORT_OK;
}

int radsort_state_logical(radsort_state* st, void* keys_out, void* payload_out, void* stream)
{
    if (!st || !st->is_setup) return RADSORT_E_INVALID;
    if ((st->count && !keys_out) || (st->g.vb && st->count && !payload_out))
        return RADSORT_E_INVALID;
    int rc = dispatch<DoLogical>(st->g.kb, st->g.vb, st, keys_out, payload_out,
                                 (hipStream_t)stream);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

int radsort_state_dims(const radsort_state* st, uint32_t* npi, uint32_t* sigma, uint32_t* nt)
{
    if (!st) return RADSORT_E_INVALID;
    if (npi) *npi = st->g.npi;
    if (sigma) *sigma = st->g.sigma;
    if (nt) *nt = st->g.nt;
    return RADSORT_OK;
}

int radsort_state_destroy(radsort_state* st)
{
    if (!st) return RADSORT_OK;
    if (st->own_ws && st->ws) (void)hipFree(st->ws);
    delete st;
    return RADSORT_OK;
}

uint64_t radsort_workspace_bytes(uint64_t n, int key_bytes, int payload_bytes, int digit_bits,
                                 const radsort_opts* opts)
{
    Geo g;
    if (make_geo(g, n, key_bytes, payload_bytes, digit_bits, opts)) return 0;
    return make_layout(g, false, g.pack_ok).total;
}

uint64_t radsort_oop_workspace_bytes(uint64_t n, int key_bytes, int payload_bytes,
                                     int digit_bits, const radsort_opts* opts)
{
    Geo g;
    if (make_geo(g, n, key_bytes, payload_bytes, digit_bits, opts)) return 0;
    return make_layout(g, true).total;
}

int radsort_workspace_error(const void* workspace, uint64_t n, int key_bytes, int payload_bytes,
                            int digit_bits, const radsort_opts* opts, int out_of_place,
                            uint32_t* error_bits, void* stream)
{
    if (error_bits) *error_bits = 0;
    if (!workspace || !opts) return RADSORT_E_INVALID;
    Geo g;
    int rc = make_geo(g, n, key_bytes, payload_bytes, digit_bits, opts);
    if (rc) return rc;
    if (n <= 1) return RADSORT_OK;  // such a call runs nothing
    // the error word lies among the small arrays at the front of every layout
    const Layout L = make_layout(g, out_of_place != 0);
    if (opts->workspace_bytes < L.ctr + 4ull * (g.nt + 1)) return RADSORT_E_NOMEM;
    hipStream_t s = (hipStream_t)stream;
    uint32_t e = 0;
    RS_HIP(hipMemcpyAsync(&e, (const uint8_t*)workspace + L.ctr + 4ull * g.nt, 4,
                          hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    if (error_bits) *error_bits = e;
    return (e & kErrOrder) ? RADSORT_E_ORDER : e ? RADSORT_E_TIMEOUT : RADSORT_OK;
}

int radsort_sort_pairs(void* keys, void* payload, uint64_t n, int key_bytes, int payload_bytes,
                       int digit_bits, const radsort_opts* opts, void* stream)
{
    int rc = check_args(keys, payload, n, payload_bytes);
    if (rc) return rc;
    Geo g;
    rc = make_geo(g, n, key_bytes, payload_bytes, digit_bits, opts);
    if (rc) return rc;
    if (n <= 1) return RADSORT_OK;
    radsort_state* st = nullptr;
    rc = state_create(&st, keys, payload, n, key_bytes, payload_bytes, digit_bits, opts, true);
    if (rc) return rc;
    // The launch form without co-residency (one workgroup per tile) is also the
    // faster one alone for blocks of up to 1024 elements (no cooperative launch per
    // round, which costs most at small n); with larger blocks the persistent form,
    // whose workgroups overlap one tile's loads with the previous tile, is faster.
    st->dynamic = (opts && (opts->flags & RADSORT_F_SHARED)) || g.b <= 1024;
    st->shared = opts && (opts->flags & RADSORT_F_SHARED);
    hipStream_t s = (hipStream_t)stream;
    const bool timing = opts && (opts->flags & RADSORT_F_TIMING);
    if (timing) g_timer.begin();
    rc = radsort_state_setup(st, s);
    for (uint32_t r = 0; !rc && r < st->g.nt; r++) rc = radsort_state_round(st, s);
    if (!rc) rc = radsort_state_finalize(st, s);
    g_timer.end();
    g_stats.timed = 0;
    g_stats.workspace_bytes = st->L.total;
    g_stats.input_bytes = n * (uint64_t)(key_bytes + payload_bytes);
    g_stats.rounds = st->g.nt;
    const bool check = opts && (opts->flags & RADSORT_F_CHECK);
    if (!rc && (check || st->own_ws)) rc = read_err(st, s, nullptr);
    radsort_state_destroy(st);  // a library-owned workspace is freed after read_err's wait
    return rc;
}

int radsort_sort(void* keys, uint64_t n, int key_bytes, int digit_bits, void* stream)
{
    return radsort_sort_pairs(keys, nullptr, n, key_bytes, 0, digit_bits, nullptr, stream);
}

int radsort_oop_sort_pairs(void* keys, void* payload, uint64_t n, int key_bytes,
                           int payload_bytes, int digit_bits, const radsort_opts* opts,
                           void* stream)
{
    int rc = check_args(keys, payload, n, payload_bytes);
    if (rc) return rc;
    Geo g;
    rc = make_geo(g, n, key_bytes, payload_bytes, digit_bits, opts);
    if (rc) return rc;
    if (n <= 1) return RADSORT_OK;
    Layout L = make_layout(g, true);
    hipStream_t s = (hipStream_t)stream;
    uint8_t* ws = nullptr;
    bool own = false;
    if (opts && opts->workspace) {
        if (opts->workspace_bytes < L.total) return RADSORT_E_NOMEM;
        ws = (uint8_t*)opts->workspace;
    } else {
        hipError_t e = hipMalloc((void**)&ws, L.total);
        if (e != hipSuccess) {
            g_last_hip = e;
            return RADSORT_E_NOMEM;
        }
        own = true;
    }
    const bool timing = opts && (opts->flags & RADSORT_F_TIMING);
    if (timing) g_timer.begin();
    // the out-of-place round runs faster in the form without co-residency (one
    // workgroup per tile) at every size and block tried, so it always takes it
    const bool dyn = true;
    rc = dispatch<DoOop>(g.kb, g.vb, keys, payload, g, L, ws, dyn, s);
    g_timer.end();
    g_stats.timed = 0;
    if (!rc) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            g_last_hip = e;
            rc = RADSORT_E_DEVICE;
        }
    }
    g_stats.workspace_bytes = L.total;
    g_stats.input_bytes = n * (uint64_t)(key_bytes + payload_bytes);
    g_stats.rounds = g.nt;
    const bool check = opts && (opts->flags & RADSORT_F_CHECK);
    if (!rc && (check || own)) {
        uint32_t e = 0;
        hipError_t he = hipMemcpyAsync(&e, ws + L.ctr + 4ull * g.nt, 4, hipMemcpyDeviceToHost, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);
        if (he != hipSuccess) {
            g_last_hip = he;
            rc = RADSORT_E_DEVICE;
        } else if (e) {
            rc = RADSORT_E_TIMEOUT;
        }
        g_stats.error_bits = e;
    }
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(ws);
    }
    return rc;
}

int radsort_histograms(const void* keys, uint64_t n, int key_bytes, int digit_bits,
                       uint32_t* counts, void* stream)
{
    if (!counts || (n && !keys)) return RADSORT_E_INVALID;
    Geo g;
    int rc = make_geo(g, n, key_bytes, 0, digit_bits, nullptr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = key_bytes == 4 ? launch_histograms<4>(keys, g, counts, s)
                        : launch_histograms<8>(keys, g, counts, s);
    if (rc) return rc;
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

int radsort_last_stats(radsort_stats* out)
{
    if (!out) return RADSORT_E_INVALID;
    g_timer.report(g_stats);
    *out = g_stats;
    return RADSORT_OK;
}

int radsort_copy(void* dst, const void* src, uint64_t bytes, void* stream)
{
    if (bytes && (!dst || !src)) return RADSORT_E_INVALID;
    if (((uintptr_t)dst | (uintptr_t)src) & 15) return RADSORT_E_INVALID;
    if (!bytes) return RADSORT_OK;
    const uint64_t words = bytes / 16;
    const uint32_t tail = (uint32_t)(bytes % 16);
    int dev = 0, cus = 0;
    RS_HIP(hipGetDevice(&dev));
    RS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // one workgroup of 256 threads per CU (fewer when there is less to copy): with
    // 4 words in flight per thread this is the fastest of the shapes measured on
    // MI355X (5.7 TB/s for 2 GiB; 8 workgroups per CU: 4.7 TB/s, 2: 5.5 TB/s)
    const uint64_t want = (words + 4 * 256 - 1) / (4 * 256);
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus));
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                       (u32x4*)dst, (const u32x4*)src, words,
                       (uint8_t*)dst + words * 16, (const uint8_t*)src + words * 16, tail);
    RS_HIP(hipGetLastError());
    return RADSORT_OK;
}

const char* radsort_strerror(int code)
{
    switch (code) {
    case RADSORT_OK: return "ok";
    case RADSORT_E_INVALID: return "invalid argument";
    case RADSORT_E_NOMEM: return "out of memory or workspace too small";
    case RADSORT_E_DEVICE: return hipGetErrorString(g_last_hip);
    case RADSORT_E_UNSUPPORTED: return "unsupported size or digit width";
    case RADSORT_E_TIMEOUT: return "a device-side check failed (a bounded wait gave up or an index left its range)";
    case RADSORT_E_ORDER: return "ordering check: a block was drawn before its loads were marked";
    default: return "unknown error";
    }
}

uint64_t radsort_segments_workspace_bytes(const uint64_t* offsets, uint32_t nseg, int key_bytes,
                                          int payload_bytes, const radsort_seg_tuning* tuning,
                                          const radsort_opts* opts)
{
    if (!offsets || (key_bytes != 4 && key_bytes != 8)) return 0;
    SegPlan P;
    if (make_seg_plan(P, offsets, nseg, key_bytes, payload_bytes, tuning, opts)) return 0;
    return P.total;
}

int radsort_sort_segments(void* keys, void* payload, const uint64_t* offsets,
                          const uint64_t* offsets_dev, uint32_t nseg, int key_bytes,
                          int payload_bytes, const radsort_seg_tuning* tuning,
                          const radsort_opts* opts, void* stream)
{
    if (!offsets || (nseg && !offsets_dev)) return RADSORT_E_INVALID;
    if (key_bytes != 4 && key_bytes != 8) return RADSORT_E_INVALID;
    if (payload_bytes != 0 && payload_bytes != 4 && payload_bytes != 8) return RADSORT_E_INVALID;
    if (nseg == 0 || offsets[nseg] == offsets[0]) return RADSORT_OK;
    int rc = check_args(keys, payload, offsets[nseg], payload_bytes);
    if (rc) return rc;
    SegPlan P;
    rc = make_seg_plan(P, offsets, nseg, key_bytes, payload_bytes, tuning, opts);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    uint8_t* ws = opts ? (uint8_t*)opts->workspace : nullptr;
    bool own = false;
    if (ws) {
        if (opts->workspace_bytes < P.total) return RADSORT_E_NOMEM;
    } else {
        hipError_t e = hipMalloc((void**)&ws, P.total);
        if (e != hipSuccess) {
            g_last_hip = e;
            return RADSORT_E_NOMEM;
        }
        own = true;
    }
    // [0]: small arrays, [1 + l]: lane l, [1 + kSegLanes]: the one-workgroup path,
    // [2 + kSegLanes]: its claim counter
    uint32_t* err_small = (uint32_t*)ws;
    launch_fill(err_small, 3 + kSegLanes, 0, s);
    // the lanes fork first, so that their sorts run beside the batched kernels on the
    // caller's stream; they join back at the end
    LaneStreams* L = nullptr;
    if (!P.large.empty()) {
        rc = lane_streams(&L);
        if (!rc && hipEventRecord(L->fork, s) != hipSuccess) rc = RADSORT_E_DEVICE;
        for (uint32_t l = 0; !rc && l < kSegLanes; l++)
            if (hipStreamWaitEvent(L->s[l], L->fork, 0) != hipSuccess) rc = RADSORT_E_DEVICE;
        const uint64_t kb = key_bytes, vb = payload_bytes;
        for (size_t k = 0; !rc && k < P.large.size(); k++) {
            const uint32_t i = P.large[k], l = P.lane[k];
            void* kp = (uint8_t*)keys + offsets[i] * kb;
            void* vp = payload ? (uint8_t*)payload + offsets[i] * vb : nullptr;
            rc = run_one(kp, vp, offsets[i + 1] - offsets[i], key_bytes, payload_bytes,
                         P.choice[k], ws + P.lane_off[l], P.lane_bytes[l], err_small + 1 + l,
                         L->s[l]);
        }
    }
    if (!rc && P.any_small) {
        rc = dispatch<DoSmall>(key_bytes, payload_bytes, keys, payload, offsets_dev, nseg,
                               err_small, s);
    }
    if (!rc && P.wg_count) {
        rc = dispatch<DoWg>(key_bytes, payload_bytes, keys, payload, offsets_dev, nseg, P, ws,
                            err_small + 2 + kSegLanes, err_small + 1 + kSegLanes, s);
    }
    if (L) {
        for (uint32_t l = 0; l < kSegLanes; l++) {
            if (hipEventRecord(L->join[l], L->s[l]) != hipSuccess && !rc) rc = RADSORT_E_DEVICE;
            if (hipStreamWaitEvent(s, L->join[l], 0) != hipSuccess && !rc) rc = RADSORT_E_DEVICE;
        }
    }
    g_stats.timed = 0;
    g_stats.workspace_bytes = P.total;
    g_stats.input_bytes = (offsets[nseg] - offsets[0]) * (uint64_t)(key_bytes + payload_bytes);
    const bool check = opts && (opts->flags & RADSORT_F_CHECK);
    if (!rc && (check || own)) {
        // every lane's error word and the small kernel's
        uint32_t e = 0;
        std::vector<uint32_t> words(2 + kSegLanes, 0);
        RS_HIP(hipStreamSynchronize(s));
        RS_HIP(hipMemcpy(words.data(), err_small, 4 * words.size(), hipMemcpyDeviceToHost));
        for (uint32_t w : words) e |= w;
        g_stats.error_bits = e;
        if (e) rc = RADSORT_E_TIMEOUT;
    }
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(ws);
    }
    return rc;
}

}  // extern "C"

// ---- MSD-first split (Sec. 4.3, last paragraph) ------------------------------------
//
// One Radsort round on the most significant digit, finalized, leaves the array
// grouped by that digit (stably); each group is then an independent sort over the
// remaining digits, run as one batch of arrays by radsort_sort_segments (the
// digit that is now constant in every group costs no round there).  The group
// boundaries come from the digit totals that the round's counting pass leaves in
// the last row of the super-tile table, read back to the host before finalize
// reuses that memory.
int radsort_msd_sort_pairs(void* keys, void* payload, uint64_t n, int key_bytes,
                           int payload_bytes, int digit_bits, const radsort_opts* opts,
                           void* stream)
{
    int rc = check_args(keys, payload, n, payload_bytes);
    if (rc) return rc;
    if (opts && opts->workspace) return RADSORT_E_INVALID;  // the library sizes each phase
    Geo g;
    rc = make_geo(g, n, key_bytes, payload_bytes, digit_bits, opts);
    if (rc) return rc;
    if (n <= 1) return RADSORT_OK;
    radsort_opts o = opts ? *opts : radsort_opts{};
    o.flags &= ~(uint32_t)RADSORT_F_TIMING;
    radsort_state* st = nullptr;
    rc = radsort_state_create(&st, keys, payload, n, key_bytes, payload_bytes, digit_bits, &o);
    if (rc) return rc;
    st->dynamic = (o.flags & RADSORT_F_SHARED) || g.b <= 1024;
    st->shared = o.flags & RADSORT_F_SHARED;
    st->msd_shift = (int)(g.bits * (g.nt - 1));
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint32_t> tot(g.sigma, 0);
    rc = radsort_state_setup(st, s);
    if (!rc) rc = radsort_state_round(st, s);
    if (!rc && hipMemcpyAsync(tot.data(), st->u32(st->L.stcnt) + (uint64_t)g.supers * g.sigma,
                              4ull * g.sigma, hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = RADSORT_E_DEVICE;
    if (!rc) rc = radsort_state_finalize(st, s);
    if (!rc) rc = read_err(st, s, nullptr);  // waits: the totals are on the host
    const uint64_t radsort_ws = st->L.total;
    radsort_state_destroy(st);
    if (rc) return rc;
    std::vector<uint64_t> off(g.sigma + 1, 0);
    for (uint32_t d = 0; d < g.sigma; d++) off[d + 1] = off[d] + tot[d];
    if (off[g.sigma] != n) return RADSORT_E_DEVICE;  // never for a consistent round
    uint64_t* off_dev = nullptr;
    hipError_t e = hipMalloc((void**)&off_dev, 8ull * (g.sigma + 1));
    if (e != hipSuccess) {
        g_last_hip = e;
        return RADSORT_E_NOMEM;
    }
    rc = RADSORT_OK;
    if (hipMemcpyAsync(off_dev, off.data(), 8ull * (g.sigma + 1), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        rc = RADSORT_E_DEVICE;
    radsort_opts so{};
    so.flags = o.flags & RADSORT_F_CHECK;
    if (!rc)
        rc = radsort_sort_segments(keys, payload, off.data(), off_dev, g.sigma, key_bytes,
                                   payload_bytes, nullptr, &so, stream);
    const uint64_t seg_ws = g_stats.workspace_bytes;
    (void)hipStreamSynchronize(s);  // off_dev is read by the segment kernels
    (void)hipFree(off_dev);
    g_stats.timed = 0;
    g_stats.workspace_bytes = std::max<uint64_t>(radsort_ws, seg_ws + 8ull * (g.sigma + 1));
    g_stats.input_bytes = n * (uint64_t)(key_bytes + payload_bytes);
    g_stats.rounds = g.nt;
    return rc;
}

// ---- the allocation-free entry point ----------------------------------------------
//
// radsort_sort_pairs_noalloc sorts with a workspace that is a file-scope device
// array, `scratch`, instead of a caller buffer or an allocation: each GPU the
// library runs on holds RADSORT_NOALLOC_SCRATCH_BYTES of it from the time the code
// object is loaded until the process ends.  In host code `scratch` names a host
// stand-in, never the device memory: its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that address is
// passed to kernels.  Every call on one GPU shares the array; the kernels clear
// what must start at zero (setup's fills), and calls that overlap on one GPU race.

static __device__ __align__(256) uint8_t scratch[RADSORT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices];  // device address of `scratch`, per device

// Device address of `scratch` on the current device (looked up on first use).
int scratch_address(void** out)
{
    int dev = 0;
    RS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return RADSORT_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        RS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return RADSORT_E_DEVICE;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return RADSORT_OK;
}

}  // namespace

int radsort_sort_pairs_noalloc(void* keys, void* payload, uint64_t n, int key_bytes,
                               int payload_bytes, int digit_bits, uint32_t block_elems,
                               uint32_t flags, void* stream)
{
    // timing records HIP events, which the library creates (allocates) on first use
    if (flags & RADSORT_F_TIMING) return RADSORT_E_INVALID;
    int rc = check_args(keys, payload, n, payload_bytes);
    if (rc) return rc;
    radsort_opts o{};
    o.block_elems = block_elems;
    o.flags = flags | RADSORT_F_SHARED;  // the launch forms below
    Geo g;
    rc = make_geo(g, n, key_bytes, payload_bytes, digit_bits, &o);
    if (rc) return rc;
    if (n <= 1) return RADSORT_OK;
    const Layout L = make_layout(g, false, g.pack_ok);
    if (L.total > (uint64_t)RADSORT_NOALLOC_SCRATCH_BYTES) return RADSORT_E_NOMEM;
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    radsort_state st;  // on the stack: nothing is allocated, on the host either
    st.g = g;
    st.L = L;
    st.ws = (uint8_t*)ws;
    st.own_ws = false;
    st.keys = keys;
    st.vals = payload;
    st.count = n;
    st.seq_draws = flags & RADSORT_F_SEQ_DRAWS;
    st.pack = g.pack_ok;
    // the launch forms that query no occupancy (the query's cache allocates)
    st.dynamic = true;
    st.shared = true;
    hipStream_t s = (hipStream_t)stream;
    rc = radsort_state_setup(&st, s);
    for (uint32_t r = 0; !rc && r < st.g.nt; r++) rc = radsort_state_round(&st, s);
    if (!rc) rc = radsort_state_finalize(&st, s);
    g_stats.timed = 0;
    g_stats.workspace_bytes = L.total;
    g_stats.input_bytes = n * (uint64_t)(key_bytes + payload_bytes);
    g_stats.rounds = st.g.nt;
    if (!rc && (flags & RADSORT_F_CHECK)) rc = read_err(&st, s, nullptr);
    return rc;
}

#ifdef RS_TIMELINE
// Timeline builds only (not part of include/radsort.h): later Radsort rounds write
// kTlStamps real-time stamps per tile into buf (device memory of tiles * kTlStamps
// words), each round over the previous one.
extern "C" int radsort_timeline_buffer(void* buf, uint64_t tiles)
{
    g_tl = (uint64_t*)buf;
    g_tl_tiles = buf ? tiles : 0;
    return RADSORT_OK;
}
#endif
