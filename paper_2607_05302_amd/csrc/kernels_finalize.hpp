// Parallel finalize (Alg. 7 in the parallel form sketched in Sec. 4.3: a
// parallel permutation of whole blocks, then closing the gaps the partial blocks
// leave).  Three steps:
//
//  F1  block permutation.  Logical block L moves to physical block
//      rot(L) = (L + sigma) mod n_pi: logical sigma .. sigma + floor(n/b) - 1 land
//      on the A blocks in order (their homes, as in Alg. 7 under reading G2) and
//      the at most sigma allocated blocks after them land in T.  The content of
//      physical p moves to next(p) = rot(pi^-1[p]), a permutation of the n_pi
//      physical blocks.  Its cycles are found by pointer jumping: after
//      ceil(log2 n_pi) doubling steps every node knows the smallest node of its
//      cycle (the leader) and its distance to it, hence its rank in the cycle and
//      the cycle length.  Nodes of cycles longer than one are laid out in an
//      order array, cycle after cycle by rank, and cut into jobs of S nodes.  A
//      job moves its nodes in decreasing rank (each node receives its
//      predecessor's content after its own content was read); the first node of
//      a piece of a cycle that spans jobs is saved to a temporary block first.
//      Jobs are split further by columns of the blocks.  Unallocated blocks
//      carry no data and are not copied.
//  F2  ordered compaction.  A block j then holds logical sigma + j; its used
//      elements move left by G_j, the unused tails of the partial blocks before
//      it (non-decreasing in j).  Chunks run in increasing dynamic order; a
//      chunk writes only after every chunk whose source its destination
//      overlaps has loaded.
//  F3  the blocks in T are copied to the end of A.
//
// After truncate (Alg. 8) the same steps apply with n_pi and the A blocks of the
// original array: the allocated blocks sigma .. f-1 are fewer, F1 leaves the
// blocks past f alone as unallocated, and F2 reads nothing from them.
//
// A packed state (its last round packed: every element already sits at the slot
// of its final position) needs no F2 and no F3: F1 moves each block to the home
// k_pack_homes gives it, over n_pi + sigma blocks, and k_pack_merge copies the
// slots of the at most sigma blocks (one per bucket) that do not fill a block of A
// into place.
#pragma once

#include <hip/hip_cooperative_groups.h>

#include "common.hpp"

namespace rs {

#ifndef RS_FIN_JOB
#define RS_FIN_JOB 1024
#endif
constexpr uint32_t kFinJob = RS_FIN_JOB;  // nodes per job of F1 (at most)
constexpr uint32_t kFinCols = 256;      // columns of a block moved by one F1 workgroup
constexpr uint32_t kFinDepth = 16;      // loads in flight per thread in F1
constexpr uint32_t kScanTile = 4096;    // elements per workgroup of the device scan
constexpr uint32_t kGarbage = 0x80000000u;

inline uint64_t fin_align(uint64_t x) { return (x + 255) / 256 * 256; }

// Bytes of finalize scratch: six n_pi-word arrays (two more reuse the second pi
// buffer and the block-length array, which finalize no longer needs), the scan's
// block sums, the F2 chunk flags and two temporary blocks per F1 job.
constexpr uint32_t kCompactMin = 4096;  // smallest F2 chunk (elements)

// F2 chunk flags (one per chunk) plus a counter
inline uint64_t fin_flag_words(uint32_t npi, uint64_t n)
{
    return std::max<uint64_t>(npi, n / kCompactMin + 1) + 16;
}

// Nodes per F1 job: kFinJob, or fewer (down to 16) for states of fewer than
// 64 kFinJob blocks, so that their blocks are spread over more workgroups; each
// job saves up to two head blocks, a small part of the workspace of such states.
inline uint32_t fin_job(uint32_t npi)
{
    uint32_t j = kFinJob;
    while (j > 16 && (uint64_t)j * 64 > npi) j >>= 1;
    return j;
}

// Finalize scratch; `temps`: with the two temporary blocks per job that only the
// two-kernel form of F1 uses (shared GPU, or a state the cooperative form cannot cover)
inline uint64_t fin_scratch_bytes(uint32_t npi, uint64_t n, uint32_t b, uint32_t elem_bytes,
                                  bool temps)
{
    const uint32_t job = fin_job(npi);
    uint64_t jobs = (npi + job - 1) / job;
    uint64_t sums = (npi + kScanTile - 1) / kScanTile + 1;
    return 6 * fin_align(4ull * npi) + fin_align(4 * sums) + fin_align(4 * fin_flag_words(npi, n)) +
           (temps ? fin_align(2 * jobs * (uint64_t)b * elem_bytes) : 0);
}

template <int KB, int VB>
struct FinArgs {
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    K* Ak;
    V* Av;
    K* Tk;
    V* Tv;
    uint32_t* pi;
    const uint32_t* Pidx;
    const uint32_t* Plen;
    const uint32_t* f;
    uint64_t n;
    uint32_t sigma, log2b, npi;
    uint32_t job;  // nodes per F1 job: fin_job(npi)
    uint32_t* err;
    uint8_t* scratch;
    uint32_t* spare_pi;  // the other pi buffer (n_pi words), free during finalize
    uint32_t* spare_blen;  // the block-length array (n_pi words), free during finalize
    // A packed state (its last round packed, plan_round): npi counts the sigma extra
    // blocks X too (physical npi_eq .. npi - 1), and F1 moves every logical block to
    // the home k_pack_homes gives it.  Otherwise pack is null and npi_eq = npi.
    K* Xk;
    V* Xv;
    uint32_t npi_eq;
    const uint32_t* est;   // packed: element start of each bucket
    const uint32_t* S;     // packed: first logical block of each bucket
    uint32_t* pack;        // packed: 2 sigma + 2 words (k_pack_table), else null
    // the block of physical index j: Eq. 1, or an extra block of a packed state
    __device__ K* kblock(uint32_t j) const
    {
        return j < npi_eq ? blockat(Ak, Tk, j, 2 * sigma, log2b) : Xk + ((uint64_t)(j - npi_eq) << log2b);
    }
    __device__ V* vblock(uint32_t j) const
    {
        return j < npi_eq ? blockat(Av, Tv, j, 2 * sigma, log2b) : Xv + ((uint64_t)(j - npi_eq) << log2b);
    }
};

struct FinArrays {
    uint32_t *nxt, *j0, *j1, *v0, *v1, *o0, *o1, *ord, *sums, *flags;
    uint64_t nflags;
    uint8_t* temps;
};

inline FinArrays fin_arrays(uint8_t* s, uint32_t npi, uint64_t n, uint32_t* spare_pi,
                            uint32_t* spare_blen)
{
    FinArrays a;
    uint64_t w = fin_align(4ull * npi);
    a.nxt = spare_pi;
    a.ord = spare_blen;
    a.j0 = (uint32_t*)(s + 0 * w);
    a.j1 = (uint32_t*)(s + 1 * w);
    a.v0 = (uint32_t*)(s + 2 * w);
    a.v1 = (uint32_t*)(s + 3 * w);
    a.o0 = (uint32_t*)(s + 4 * w);
    a.o1 = (uint32_t*)(s + 5 * w);
    a.sums = (uint32_t*)(s + 6 * w);
    uint64_t sums = (npi + kScanTile - 1) / kScanTile + 1;
    a.flags = (uint32_t*)(s + 6 * w + fin_align(4 * sums));
    a.nflags = fin_flag_words(npi, n);
    a.temps = s + 6 * w + fin_align(4 * sums) + fin_align(4 * a.nflags);
    return a;
}

// ---- F1: cycles of next(p) ----------------------------------------------------------

// next(pi[L]) = rot(L); the top bit marks a node whose content is unallocated.
// Doubling state: J = next, (V, O) = (p, 0).
// homes (packed states): next(pi[L]) = homes[L] and its top bit marks no data.
__global__ void k_fin_init(const uint32_t* __restrict__ pi, const uint32_t* __restrict__ f_ptr,
                           uint32_t sigma, uint32_t npi, uint32_t* __restrict__ nxt,
                           uint32_t* __restrict__ J, uint32_t* __restrict__ V,
                           uint32_t* __restrict__ O, const uint32_t* __restrict__ homes)
{
    const uint32_t f = *f_ptr;
    for (uint32_t L = blockIdx.x * blockDim.x + threadIdx.x; L < npi;
         L += gridDim.x * blockDim.x) {
        const uint32_t p = pi[L];
        if (p >= npi) continue;  // never for a permutation
        uint32_t to = L + sigma < npi ? L + sigma : L + sigma - npi;
        bool garbage = L < sigma || L >= f;
        if (homes) {
            to = homes[L] & ~kGarbage;
            garbage = homes[L] & kGarbage;
            if (to >= npi) to = p;  // never for a consistent table
        }
        nxt[p] = to | (garbage ? kGarbage : 0u);
        J[p] = to;
        V[p] = p;
        O[p] = 0;
    }
}

// Pointer jumping, two doubling steps per launch.  (V, O) of node p is the
// smallest node within the window of its next 2^k successors (p included) and the
// distance to its first occurrence; J(p) is the node 2^k steps on.  One launch
// takes the window to 2^(k+2) from the four windows that start at p, J(p), J(J(p))
// and J(J(J(p))), in that order, so that the first occurrence of the smallest node
// wins.
__global__ void k_fin_jump4(const uint32_t* __restrict__ Ji, const uint32_t* __restrict__ Vi,
                            const uint32_t* __restrict__ Oi, uint32_t* __restrict__ Jo,
                            uint32_t* __restrict__ Vo, uint32_t* __restrict__ Oo, uint32_t npi,
                            uint32_t window)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npi;
         p += gridDim.x * blockDim.x) {
        uint32_t v = Vi[p], o = Oi[p], q = p;
#pragma unroll
        for (uint32_t k = 1; k < 4; k++) {
            uint32_t qn = Ji[q];
            if (qn >= npi) qn = q;  // never for a permutation
            q = qn;
            const uint32_t v2 = Vi[q];
            if (v2 < v) {
                v = v2;
                o = Oi[q] + k * window;
            }
        }
        uint32_t qn = Ji[q];
        if (qn >= npi) qn = q;
        Vo[p] = v;
        Oo[p] = o;
        Jo[p] = qn;
    }
}

// rank of p in its cycle (0 at the leader) and the cycle length; the scan input
// is the cycle length at leaders of cycles longer than one.
__global__ void k_fin_rank(const uint32_t* __restrict__ nxt, const uint32_t* __restrict__ V,
                           const uint32_t* __restrict__ O, uint32_t* __restrict__ rank,
                           uint32_t* __restrict__ clen, uint32_t* __restrict__ scan_in,
                           uint32_t npi)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npi;
         p += gridDim.x * blockDim.x) {
        const uint32_t l = V[p] < npi ? V[p] : p;
        uint32_t ln = nxt[l] & ~kGarbage;
        if (ln >= npi) ln = l;  // never for a permutation
        const uint32_t len = ln == l ? 1u : O[ln] + 1u;
        rank[p] = p == l ? 0u : len - O[p];
        clen[p] = len;
        scan_in[p] = (p == l && len > 1) ? len : 0u;
    }
}

__global__ void k_fin_order(const uint32_t* __restrict__ nxt, const uint32_t* __restrict__ V,
                            const uint32_t* __restrict__ rank, const uint32_t* __restrict__ clen,
                            const uint32_t* __restrict__ base, uint32_t* __restrict__ ord,
                            uint32_t npi)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npi;
         p += gridDim.x * blockDim.x) {
        if (clen[p] > 1 && V[p] < npi) {
            const uint32_t at = base[V[p]] + rank[p];
            if (at < npi) ord[at] = p | (nxt[p] & kGarbage);
        }
    }
}

// The whole preparation of F1 (next, the doubling steps, ranks, cycle lengths,
// the scan of the leaders' cycle lengths and the order array) plus the gap
// prefix of F2 and the clearing of F2's chunk flags, in one workgroup with the
// doubling state in LDS, for n_pi <= kFinSmallNodes.  Same results as
// k_fin_init .. k_fin_order and k_fin_gaps: rank, clen, ord and *M_out (the
// number of nodes to move) in global memory for k_fin_save / k_fin_move, and
// gap[0 .. sigma] for F2 / F3.
constexpr uint32_t kFinSmallNodes = 8192;
template <int NT>
__global__ __launch_bounds__(NT) void k_fin_prep_small(
    const uint32_t* __restrict__ pi, const uint32_t* __restrict__ f_ptr,
    const uint32_t* __restrict__ Pidx, const uint32_t* __restrict__ Plen, uint32_t sigma,
    uint32_t log2b, uint32_t npi, uint32_t* __restrict__ rank, uint32_t* __restrict__ clen,
    uint32_t* __restrict__ ord, uint32_t* __restrict__ M_out, uint32_t* __restrict__ gap,
    uint32_t* __restrict__ flags, uint64_t nflags, uint32_t* __restrict__ err,
    const uint32_t* __restrict__ homes)
{
    constexpr uint32_t PER = kFinSmallNodes / NT;  // nodes per thread
    __shared__ uint32_t nx[kFinSmallNodes], J[kFinSmallNodes], Vs[kFinSmallNodes],
        Os[kFinSmallNodes];
    __shared__ uint32_t tmp[NT / 64 + 1];
    const uint32_t tid = threadIdx.x, f = *f_ptr;
    if (npi > kFinSmallNodes) {  // never for a call made by the library
        if (tid == 0) raise_error(err, kErrBounds);
        return;
    }
    for (uint64_t i = tid; i < nflags; i += NT) flags[i] = 0;
    // next(pi[L]) = rot(L), garbage bit for unallocated L; J = next, (V, O) = (p, 0)
    for (uint32_t L = tid; L < npi; L += NT) {
        uint32_t p = pi[L];
        if (p >= npi) {  // never for a permutation
            raise_error(err, kErrBounds);
            p = L;
        }
        uint32_t to = L + sigma < npi ? L + sigma : L + sigma - npi;
        uint32_t gb = (L < sigma || L >= f) ? kGarbage : 0u;
        if (homes) {  // packed state
            to = homes[L] & ~kGarbage;
            gb = homes[L] & kGarbage;
            if (to >= npi) to = p;  // never for a consistent table
        }
        nx[p] = to | gb;
        J[p] = to;
        Vs[p] = p;
        Os[p] = 0;
    }
    __syncthreads();
    // doubling: (V, O) = smallest node within 2^k successors and its distance
    for (uint32_t w = 1; w < npi; w <<= 1) {
        uint32_t jn[PER], vn[PER], on[PER];
#pragma unroll
        for (uint32_t k = 0; k < PER; k++) {
            const uint32_t p = tid + k * NT;
            if (p < npi) {
                uint32_t q = J[p];
                if (q >= npi) q = p;
                uint32_t v = Vs[p], o = Os[p];
                const uint32_t v2 = Vs[q];
                if (v2 < v) {
                    v = v2;
                    o = Os[q] + w;
                }
                jn[k] = J[q];
                vn[k] = v;
                on[k] = o;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < PER; k++) {
            const uint32_t p = tid + k * NT;
            if (p < npi) {
                J[p] = jn[k];
                Vs[p] = vn[k];
                Os[p] = on[k];
            }
        }
        __syncthreads();
    }
    // rank in the cycle (0 at the leader), cycle length, scan input at leaders
    uint32_t rk[PER], ln[PER];
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
        const uint32_t p = tid + k * NT;
        rk[k] = ln[k] = 0;
        if (p < npi) {
            const uint32_t l = Vs[p] < npi ? Vs[p] : p;
            uint32_t lnx = nx[l] & ~kGarbage;
            if (lnx >= npi) lnx = l;
            const uint32_t len = lnx == l ? 1u : Os[lnx] + 1u;
            rk[k] = p == l ? 0u : len - Os[p];
            ln[k] = len;
        }
    }
    __syncthreads();  // J is free: it takes the scan input
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
        const uint32_t p = tid + k * NT;
        if (p < npi) {
            J[p] = (rk[k] == 0 && ln[k] > 1) ? ln[k] : 0u;
            rank[p] = rk[k];
            clen[p] = ln[k];
        }
    }
    __syncthreads();
    const uint32_t M = block_excl_scan<NT>(J, npi, tmp);  // J[leader] = its cycle's base
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
        const uint32_t p = tid + k * NT;
        if (p < npi && ln[k] > 1 && Vs[p] < npi) {
            const uint32_t at = J[Vs[p]] + rk[k];
            if (at < npi) ord[at] = p | (nx[p] & kGarbage);
        }
    }
    if (tid == 0) *M_out = M;
    // F2's gap prefix: unused room of the partial blocks of P before each entry
    __syncthreads();  // Os is free
    const uint32_t b = 1u << log2b;
    for (uint32_t i = tid; i < sigma; i += NT) Os[i] = Pidx[i] < npi ? b - Plen[i] : 0u;
    __syncthreads();
    const uint32_t total = block_excl_scan<NT>(Os, sigma, tmp);
    for (uint32_t i = tid; i < sigma; i += NT) gap[i] = Os[i];
    if (tid == 0) gap[sigma] = total;
}

// ---- device exclusive scan of n_pi words (three passes) ------------------------------

__global__ __launch_bounds__(256) void k_scan_tiles(uint32_t* a, uint32_t count, uint32_t* sums)
{
    __shared__ uint32_t s[kScanTile];
    __shared__ uint32_t tmp[5];
    const uint32_t base = blockIdx.x * kScanTile;
    for (uint32_t i = threadIdx.x; i < kScanTile; i += 256)
        s[i] = base + i < count ? a[base + i] : 0u;
    __syncthreads();
    uint32_t total = block_excl_scan<256>(s, kScanTile, tmp);
    for (uint32_t i = threadIdx.x; i < kScanTile; i += 256)
        if (base + i < count) a[base + i] = s[i];
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_sums(uint32_t* sums, uint32_t count)
{
    __shared__ uint32_t tmp[5];
    __shared__ uint32_t s[kScanTile];
    // count <= kScanTile: n_pi < 2^24 words per scan tile level is enough here
    for (uint32_t i = threadIdx.x; i < kScanTile; i += 256) s[i] = i < count ? sums[i] : 0u;
    __syncthreads();
    uint32_t total = block_excl_scan<256>(s, kScanTile, tmp);
    for (uint32_t i = threadIdx.x; i < count; i += 256) sums[i] = s[i];
    if (threadIdx.x == 0) sums[count] = total;
}

__global__ void k_scan_add(uint32_t* a, uint32_t count, const uint32_t* sums)
{
    const uint32_t add = sums[blockIdx.x];
    const uint32_t base = blockIdx.x * kScanTile;
    for (uint32_t i = threadIdx.x; i < kScanTile; i += blockDim.x)
        if (base + i < count) a[base + i] += add;
}

// ---- F1 jobs ---------------------------------------------------------------------------

// The pieces of job j whose first node is overwritten by another job: the piece
// at the job start (slot 2j) and the last piece if it starts inside the job and
// continues after it (slot 2j + 1).  Returns the node (with garbage bit) or ~0.
__device__ __forceinline__ void job_heads(const uint32_t* ord, const uint32_t* rank,
                                          const uint32_t* clen, uint32_t j, uint32_t job,
                                          uint32_t M, uint32_t npi, uint32_t& h0, uint32_t& h1)
{
    const uint32_t i0 = j * job, i1 = min(M, i0 + job);
    h0 = h1 = ~0u;
    if (i1 <= i0) return;
    const uint32_t p0 = ord[i0] & ~kGarbage;
    const uint32_t pl0 = ord[i1 - 1] & ~kGarbage;
    if (p0 >= npi || pl0 >= npi) return;
    const uint32_t b0 = i0 - rank[p0];
    if (rank[p0] != 0 || b0 + clen[p0] > i1) h0 = ord[i0];
    const uint32_t pl = ord[i1 - 1] & ~kGarbage;
    const uint32_t bl = (i1 - 1) - rank[pl];
    if (bl > i0 && bl < i1 && bl + clen[pl] > i1) h1 = ord[bl];
}

template <typename X>
__device__ __forceinline__ void copy_block_cols(X* dst, const X* src, uint32_t b)
{
    for (uint32_t c = threadIdx.x; c < b; c += blockDim.x) dst[c] = src[c];
}

// Saves the first node of every piece that another job overwrites.
template <int KB, int VB>
__global__ __launch_bounds__(256) void k_fin_save(FinArgs<KB, VB> a, FinArrays f,
                                                  const uint32_t* rank, const uint32_t* clen,
                                                  const uint32_t* M_ptr)
{
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    const uint32_t M = min(*M_ptr, a.npi), j = blockIdx.x, b = 1u << a.log2b;
    if (j * a.job >= M) return;
    uint32_t h[2];
    job_heads(f.ord, rank, clen, j, a.job, M, a.npi, h[0], h[1]);
    K* tk = (K*)f.temps;
    V* tv = (V*)(f.temps + 2ull * ((a.npi + a.job - 1) / a.job) * b * KB);
    for (int s = 0; s < 2; s++) {
        if (h[s] == ~0u || (h[s] & kGarbage)) continue;
        if (h[s] >= a.npi) {  // never for a consistent order array
            if (threadIdx.x == 0) raise_error(a.err, kErrBounds);
            continue;
        }
        const uint64_t slot = 2ull * j + s;
        copy_block_cols(tk + (slot << a.log2b), a.kblock(h[s]), b);
        if constexpr (VB != 0)
            copy_block_cols(tv + (slot << a.log2b), a.vblock(h[s]), b);
    }
}

// VEC consecutive columns of a block, moved by one thread as one wide access
// (VEC = 4: 16 bytes for 4-byte elements), held in a vector register group.
template <typename T, int VEC> struct Cols {
    typedef T type __attribute__((ext_vector_type(VEC)));
};
template <typename T> struct Cols<T, 1> {
    using type = T;
};

// Moves one column slice of one job: grid = jobs x (b / (kFinCols VEC)).  Thread
// t of slice y moves columns (y kFinCols + t) VEC .. + VEC - 1 of every block of
// the job; VEC = 4 needs the caller's arrays 16-byte aligned (b >= 64 keeps every
// block start aligned then), else VEC = 1.
template <int KB, int VB, int VEC>
__global__ __launch_bounds__(kFinCols) void k_fin_move(FinArgs<KB, VB> a, FinArrays f,
                                                      const uint32_t* rank, const uint32_t* clen,
                                                      const uint32_t* M_ptr)
{
    using K = typename Cols<typename UInt<KB>::T, VEC>::type;
    using V = typename Cols<typename Payload<VB>::T, VEC>::type;
    using KE = typename UInt<KB>::T;
    using VE = typename Payload<VB>::T;
    const uint32_t M = min(*M_ptr, a.npi), j = blockIdx.x, b = 1u << a.log2b;
    const uint32_t i0 = j * a.job;
    if (i0 >= M) return;
    const uint32_t i1 = min(M, i0 + a.job);
    const uint32_t col = (blockIdx.y * kFinCols + threadIdx.x) * VEC;
    const bool active = col < b;  // b is a multiple of VEC
    const uint32_t log2b = a.log2b;
    // loads in flight per thread: about 512 bytes of registers
    constexpr uint32_t DEPTH = VEC == 1 ? kFinDepth : (KB + VB <= 8 ? 16u : 8u);
    const KE* tk = (const KE*)f.temps;
    const VE* tv = (const VE*)(f.temps + 2ull * ((a.npi + a.job - 1) / a.job) * b * KB);
    // the job's part of the order array, and the whole cycle of a piece that
    // crosses the job's start or end is read from global memory
    __shared__ uint32_t sord[kFinJob];
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += kFinCols) sord[i - i0] = f.ord[i];
    __syncthreads();
    auto ord_at = [&](uint32_t i) { return i >= i0 && i < i1 ? sord[i - i0] : f.ord[i]; };

    // node ids come from the order array; an id outside [0, n_pi) is clamped to a
    // T block (only possible for a corrupt state, which also raises an error)
    auto safe = [&](uint32_t node) { return node < a.npi ? node : 0u; };
    auto addr_k = [&](uint32_t node) {
        return (K*)(a.kblock(safe(node)) + col);
    };
    auto addr_v = [&](uint32_t node) {
        return (V*)(a.vblock(safe(node)) + col);
    };

    uint32_t i = i0;
    while (i < i1) {
        const uint32_t p = sord[i - i0] & ~kGarbage;
        if (p >= a.npi) {  // never for a consistent order array
            if (threadIdx.x == 0) raise_error(a.err, kErrBounds);
            return;
        }
        const uint32_t r = rank[p], L = clen[p], cb = i - r;  // cycle base in ord
        if (r >= L || cb + L > M) {
            if (threadIdx.x == 0) raise_error(a.err, kErrBounds);
            return;
        }
        const uint32_t e = min(i1, cb + L);                   // piece covers ord[i .. e)
        const uint32_t ra = r, rb = r + (e - i);
        const bool whole = ra == 0 && rb == L;
        // the head's content: from a register (whole cycle) or a saved block
        K hk{};
        V hv{};
        const uint32_t head = sord[i - i0];
        const bool head_garbage = head & kGarbage;
        if (active && !head_garbage) {
            if (whole) {
                hk = *addr_k(head & ~kGarbage);
                if constexpr (VB != 0) hv = *addr_v(head & ~kGarbage);
            } else {
                const uint64_t slot = 2ull * j + (i == i0 ? 0 : 1);
                hk = *(const K*)(tk + (slot << log2b) + col);
                if constexpr (VB != 0) hv = *(const V*)(tv + (slot << log2b) + col);
            }
        }
        // node(x + 1 mod L) <- node(x) for x = rb-1 down to ra+1, in batches
        uint32_t x = rb;  // next source rank + 1
        while (x > ra + 1) {
            const uint32_t cnt = min(DEPTH, x - (ra + 1));
            K bk[DEPTH];
            V bv[DEPTH];
            uint32_t src[DEPTH + 1];
#pragma unroll
            for (uint32_t u = 0; u < DEPTH; u++) {
                if (u < cnt) {
                    src[u] = ord_at(cb + x - 1 - u);
                    if (active && !(src[u] & kGarbage)) {
                        bk[u] = *addr_k(src[u] & ~kGarbage);
                        if constexpr (VB != 0) bv[u] = *addr_v(src[u] & ~kGarbage);
                    }
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < DEPTH; u++) {
                if (u < cnt) {
                    const uint32_t rd = x - u;  // destination rank (mod L)
                    const uint32_t dst = ord_at(cb + (rd == L ? 0 : rd)) & ~kGarbage;
                    if (active && !(src[u] & kGarbage)) {
                        *addr_k(dst) = bk[u];
                        if constexpr (VB != 0) *addr_v(dst) = bv[u];
                    }
                }
            }
            x -= cnt;
        }
        // node(ra + 1 mod L) <- head
        {
            const uint32_t rd = ra + 1;
            const uint32_t dst = ord_at(cb + (rd == L ? 0 : rd)) & ~kGarbage;
            if (active && !head_garbage) {
                *addr_k(dst) = hk;
                if constexpr (VB != 0) *addr_v(dst) = hv;
            }
        }
        i = e;
    }
}

// F1 in one cooperative launch (one workgroup of kFinLdsThreads per compute unit,
// all resident): workgroup g owns jobs g jpw .. g jpw + jpw - 1 of `job` nodes
// each.  It first copies the heads of its jobs' pieces (the nodes another job
// overwrites, as k_fin_save picks them) into its LDS, then every workgroup meets
// at a grid barrier, then each moves its jobs' nodes as k_fin_move does, taking
// the heads from LDS.  Jobs can be many and short without any temporary block in
// global memory: jpw * 2 heads of b (s_k + s_v) bytes must fit the dynamic LDS.
constexpr uint32_t kFinLdsThreads = 512;
constexpr uint32_t kFinLdsBytes = 128u << 10;  // dynamic LDS for saved heads
constexpr uint32_t kFinLdsJobMax = 4096;       // nodes per job held in LDS

// The cooperative form's shape for n_pi nodes on lds_grid workgroups (one per
// compute unit): jpw jobs per workgroup, up to 8 as the LDS holds their heads
// (2 jpw blocks of b records), fewer for small states so that their jobs of 16
// nodes still spread over the workgroups; jobs of at most kFinLdsJobMax nodes.
// covers: every node falls into one of the grid's jobs (else the two-kernel
// form of F1 must run).
struct FinCoop {
    uint32_t jpw = 0, job = 0, grid = 0;
    bool covers = false;
};
inline FinCoop fin_coop(uint32_t npi, uint32_t b, uint32_t elem_bytes, uint32_t lds_grid)
{
    FinCoop c;
    if (!lds_grid) return c;
    const uint64_t head_bytes = (uint64_t)b * elem_bytes;
    const uint64_t jpw_fill = (npi + 16ull * lds_grid - 1) / (16ull * lds_grid);
    c.jpw = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(8, kFinLdsBytes / (2 * head_bytes)),
                                         std::max<uint64_t>(1, jpw_fill));
    if (!c.jpw) return c;
    uint64_t job = (npi + (uint64_t)lds_grid * c.jpw - 1) / ((uint64_t)lds_grid * c.jpw);
    c.job = (uint32_t)std::max<uint64_t>(16, std::min<uint64_t>(job, kFinLdsJobMax));
    c.grid = (uint32_t)std::min<uint64_t>(lds_grid, (npi + (uint64_t)c.job * c.jpw - 1) /
                                                        ((uint64_t)c.job * c.jpw));
    c.covers = (uint64_t)c.grid * c.jpw * c.job >= npi;
    return c;
}

template <int KB, int VB, int VEC>
__global__ __launch_bounds__(kFinLdsThreads) void k_fin_move_lds(
    FinArgs<KB, VB> a, FinArrays f, const uint32_t* rank, const uint32_t* clen,
    const uint32_t* M_ptr, uint32_t job, uint32_t jpw)
{
    using K = typename Cols<typename UInt<KB>::T, VEC>::type;
    using V = typename Cols<typename Payload<VB>::T, VEC>::type;
    using KE = typename UInt<KB>::T;
    using VE = typename Payload<VB>::T;
    extern __shared__ __align__(16) uint8_t saved[];
    __shared__ uint32_t sord[kFinLdsJobMax];
    // loads in flight per thread (twice the threads of k_fin_move, half the depth)
    constexpr uint32_t DEPTH = VEC == 1 ? kFinDepth : (KB + VB <= 8 ? 8u : 4u);
    const uint32_t M = min(*M_ptr, a.npi), b = 1u << a.log2b, log2b = a.log2b;
    const uint32_t tid = threadIdx.x;
    KE* const hk_base = (KE*)saved;                                   // 2 jpw key blocks
    VE* const hv_base = (VE*)(saved + 2ull * jpw * ((uint64_t)b * KB)); // then payload
    auto safe = [&](uint32_t node) { return node < a.npi ? node : 0u; };

    // ---- save the heads of every job of this workgroup -------------------------------
    for (uint32_t k = 0; k < jpw; k++) {
        const uint32_t j = blockIdx.x * jpw + k;
        if ((uint64_t)j * job >= M) break;
        uint32_t h[2];
        job_heads(f.ord, rank, clen, j, job, M, a.npi, h[0], h[1]);
        for (int q = 0; q < 2; q++) {
            if (h[q] == ~0u || (h[q] & kGarbage)) continue;
            if (h[q] >= a.npi) {  // never for a consistent order array
                if (tid == 0) raise_error(a.err, kErrBounds);
                continue;
            }
            const uint64_t slot = 2ull * k + q;
            const KE* src = a.kblock(h[q]);
            for (uint32_t c = tid; c < b; c += kFinLdsThreads) hk_base[(slot << log2b) + c] = src[c];
            if constexpr (VB != 0) {
                const VE* sv = a.vblock(h[q]);
                for (uint32_t c = tid; c < b; c += kFinLdsThreads)
                    hv_base[(slot << log2b) + c] = sv[c];
            }
        }
    }
    // every head of every job is read before any job writes a block
    __builtin_amdgcn_s_waitcnt(0);
    cooperative_groups::this_grid().sync();

    // ---- move the jobs' nodes ------------------------------------------------------------
    for (uint32_t k = 0; k < jpw; k++) {
        const uint32_t j = blockIdx.x * jpw + k;
        const uint32_t i0 = j * job;
        if (i0 >= M) break;
        const uint32_t i1 = min(M, i0 + job);
        __syncthreads();  // the previous job is done with sord
        for (uint32_t i = i0 + tid; i < i1; i += kFinLdsThreads) sord[i - i0] = f.ord[i];
        __syncthreads();
        auto ord_at = [&](uint32_t i) { return i >= i0 && i < i1 ? sord[i - i0] : f.ord[i]; };
        for (uint32_t col0 = 0; col0 < b; col0 += kFinLdsThreads * VEC) {
            const uint32_t col = col0 + tid * VEC;
            const bool active = col < b;  // b is a multiple of VEC
            auto addr_k = [&](uint32_t node) {
                return (K*)(a.kblock(safe(node)) + col);
            };
            auto addr_v = [&](uint32_t node) {
                return (V*)(a.vblock(safe(node)) + col);
            };
            uint32_t i = i0;
            while (i < i1) {
                const uint32_t p = sord[i - i0] & ~kGarbage;
                if (p >= a.npi) {  // never for a consistent order array
                    if (tid == 0) raise_error(a.err, kErrBounds);
                    return;
                }
                const uint32_t r = rank[p], L = clen[p], cb = i - r;  // cycle base in ord
                if (r >= L || cb + L > M) {
                    if (tid == 0) raise_error(a.err, kErrBounds);
                    return;
                }
                const uint32_t e = min(i1, cb + L);  // piece covers ord[i .. e)
                const uint32_t ra = r, rb = r + (e - i);
                const bool whole = ra == 0 && rb == L;
                K hk{};
                V hv{};
                const uint32_t head = sord[i - i0];
                const bool head_garbage = head & kGarbage;
                if (active && !head_garbage) {
                    if (whole) {
                        hk = *addr_k(head & ~kGarbage);
                        if constexpr (VB != 0) hv = *addr_v(head & ~kGarbage);
                    } else {
                        const uint64_t slot = 2ull * k + (i == i0 ? 0 : 1);
                        hk = *(const K*)(hk_base + (slot << log2b) + col);
                        if constexpr (VB != 0) hv = *(const V*)(hv_base + (slot << log2b) + col);
                    }
                }
                // node(x + 1 mod L) <- node(x) for x = rb-1 down to ra+1, in batches
                uint32_t x = rb;
                while (x > ra + 1) {
                    const uint32_t cnt = min(DEPTH, x - (ra + 1));
                    K bk[DEPTH];
                    V bv[DEPTH];
                    uint32_t src[DEPTH];
#pragma unroll
                    for (uint32_t u = 0; u < DEPTH; u++) {
                        if (u < cnt) {
                            src[u] = ord_at(cb + x - 1 - u);
                            if (active && !(src[u] & kGarbage)) {
                                bk[u] = *addr_k(src[u] & ~kGarbage);
                                if constexpr (VB != 0) bv[u] = *addr_v(src[u] & ~kGarbage);
                            }
                        }
                    }
#pragma unroll
                    for (uint32_t u = 0; u < DEPTH; u++) {
                        if (u < cnt) {
                            const uint32_t rd = x - u;  // destination rank (mod L)
                            const uint32_t dst = ord_at(cb + (rd == L ? 0 : rd)) & ~kGarbage;
                            if (active && !(src[u] & kGarbage)) {
                                *addr_k(dst) = bk[u];
                                if constexpr (VB != 0) *addr_v(dst) = bv[u];
                            }
                        }
                    }
                    x -= cnt;
                }
                // node(ra + 1 mod L) <- head
                {
                    const uint32_t rd = ra + 1;
                    const uint32_t dst = ord_at(cb + (rd == L ? 0 : rd)) & ~kGarbage;
                    if (active && !head_garbage) {
                        *addr_k(dst) = hk;
                        if constexpr (VB != 0) *addr_v(dst) = hv;
                    }
                }
                i = e;
            }
        }
    }
}

// ---- finalize of a packed state ------------------------------------------------------
//
// After the packed round, block q of bucket d holds the ranks whose final positions
// lie in block g = floor(est[d] / b) + q of A, each at the slot it has there: slots
// lo .. hi - 1 with lo = est[d] mod b for q = 0, else 0.  So the data needs no gap
// closed, only blocks moved: every block g < floor(n/b) of A is the home of its
// "primary", the block whose slots reach the end of g (exactly one per g).  Each
// other block with data is the last block of its bucket, ending inside a block of
// A or lying in the partial tail [floor(n/b) b, n); it moves to a spare block (of
// T or X) and is copied into place afterwards (k_pack_merge), its slots only, over
// the garbage the primary brought into those slots.  Blocks without data (the
// head start, the unallocated ones, a bucket's empty head or empty last block)
// take the spare blocks left.  Spare k is physical k for k < 2 sigma, else
// npi_eq + k - 2 sigma.

__device__ __forceinline__ uint32_t pack_spare(uint32_t k, uint32_t sigma, uint32_t npi_eq)
{
    return k < 2 * sigma ? k : npi_eq + (k - 2 * sigma);
}

// The bucket table (one workgroup): tab[d] = rank of bucket d's spare block among
// those of buckets before it (~0: none), tab[sigma + d] = rank of its empty block
// (~0: none), tab[2 sigma] and tab[2 sigma + 1] the totals.
template <int NT>
__global__ __launch_bounds__(NT) void k_pack_table(const uint32_t* __restrict__ est, uint64_t n,
                                                   uint32_t sigma, uint32_t log2b,
                                                   uint32_t* __restrict__ tab)
{
    extern __shared__ uint32_t sh[];  // 2 sigma words
    __shared__ uint32_t tmp[NT / 64 + 1];
    const uint32_t b = 1u << log2b;
    const uint64_t nA = n >> log2b;
    for (uint32_t d = threadIdx.x; d < sigma; d += NT) {
        const uint64_t e0 = est[d], e1 = d + 1 < sigma ? est[d + 1] : n;
        const uint64_t c = e1 > e0 ? e1 - e0 : 0, o = e0 & (b - 1);
        bool spare = false;
        if (c) {
            const uint64_t ql = (o + c - 1) >> log2b, gl = (e0 >> log2b) + ql;
            const uint64_t hl = o + c - (ql << log2b);
            spare = gl >= nA || hl < b;
        }
        sh[d] = spare;
        sh[sigma + d] = c == 0 || ((o + c) & (b - 1)) == 0;
    }
    __syncthreads();
    const uint32_t ns = block_excl_scan<NT>(sh, sigma, tmp);
    const uint32_t ne = block_excl_scan<NT>(sh + sigma, sigma, tmp);
    for (uint32_t d = threadIdx.x; d < sigma; d += NT) {
        const uint64_t e0 = est[d], e1 = d + 1 < sigma ? est[d + 1] : n;
        const uint64_t c = e1 > e0 ? e1 - e0 : 0, o = e0 & (b - 1);
        bool spare = false;
        if (c) {
            const uint64_t ql = (o + c - 1) >> log2b, gl = (e0 >> log2b) + ql;
            const uint64_t hl = o + c - (ql << log2b);
            spare = gl >= nA || hl < b;
        }
        const bool empty = c == 0 || ((o + c) & (b - 1)) == 0;
        tab[d] = spare ? sh[d] : ~0u;
        tab[sigma + d] = empty ? sh[sigma + d] : ~0u;
    }
    if (threadIdx.x == 0) {
        tab[2 * sigma] = ns;
        tab[2 * sigma + 1] = ne;
    }
}

// homes[L] for every logical block L < npi (npi = npi_eq + sigma): its primary's A
// block, a spare block, or (top bit set) a spare block for a block without data.
__global__ void k_pack_homes(const uint32_t* __restrict__ S, const uint32_t* __restrict__ est,
                             const uint32_t* __restrict__ f_ptr, const uint32_t* __restrict__ tab,
                             uint64_t n, uint32_t sigma, uint32_t log2b, uint32_t npi_eq,
                             uint32_t npi, uint32_t* __restrict__ homes,
                             uint32_t* __restrict__ err)
{
    const uint32_t b = 1u << log2b, f = min(*f_ptr, npi);
    const uint64_t nA = n >> log2b;
    const uint32_t ns = tab[2 * sigma], ne = tab[2 * sigma + 1];
    for (uint32_t L = blockIdx.x * blockDim.x + threadIdx.x; L < npi;
         L += gridDim.x * blockDim.x) {
        uint32_t h;
        if (L < sigma) {
            h = pack_spare(ns + L, sigma, npi_eq) | kGarbage;
        } else if (L >= f) {
            h = pack_spare(ns + sigma + ne + (L - f), sigma, npi_eq) | kGarbage;
        } else {
            uint32_t lo_d = 0, hi_d = sigma;  // the last bucket d with S[d] <= L
            while (hi_d - lo_d > 1) {
                const uint32_t mid = (lo_d + hi_d) >> 1;
                if (S[mid] <= L) lo_d = mid;
                else hi_d = mid;
            }
            const uint32_t d = lo_d, q = L - S[d];
            const uint64_t e0 = est[d], e1 = d + 1 < sigma ? est[d + 1] : n;
            const uint64_t c = e1 > e0 ? e1 - e0 : 0, o = e0 & (b - 1);
            const uint64_t start = (uint64_t)q << log2b, g = (e0 >> log2b) + q;
            const uint64_t lo = q == 0 ? o : 0;
            const uint64_t hi = o + c > start ? min<uint64_t>(b, o + c - start) : 0;
            if (hi <= lo) {
                const uint32_t r = tab[sigma + d];
                h = pack_spare(ns + sigma + (r == ~0u ? 0 : r), sigma, npi_eq) | kGarbage;
                if (r == ~0u) raise_error(err, kErrBounds);  // never for a consistent plan
            } else if (g < nA && hi == b) {
                h = 2 * sigma + (uint32_t)g;
            } else {
                const uint32_t r = tab[d];
                h = pack_spare(r == ~0u ? 0 : r, sigma, npi_eq);
                if (r == ~0u) raise_error(err, kErrBounds);  // never for a consistent plan
            }
        }
        homes[L] = h;
    }
}

// After F1: workgroup d copies the slots of bucket d's spare block (if it has one)
// from that block into A.
template <int KB, int VB>
__global__ __launch_bounds__(256) void k_pack_merge(FinArgs<KB, VB> a)
{
    const uint32_t d = blockIdx.x, sigma = a.sigma, log2b = a.log2b, b = 1u << log2b;
    const uint32_t r = a.pack[d];
    if (r == ~0u) return;
    const uint64_t e0 = a.est[d], e1 = d + 1 < sigma ? a.est[d + 1] : a.n;
    const uint64_t c = e1 > e0 ? e1 - e0 : 0, o = e0 & (b - 1);
    if (!c) return;
    const uint64_t ql = (o + c - 1) >> log2b, g = (e0 >> log2b) + ql;
    const uint64_t lo = ql == 0 ? o : 0, hi = o + c - (ql << log2b);
    const uint64_t base = g << log2b;
    if (base + hi > a.n || hi > b) {  // never for a consistent plan
        if (threadIdx.x == 0) raise_error(a.err, kErrBounds);
        return;
    }
    const uint32_t from = pack_spare(r, sigma, a.npi_eq);
    const auto* sk = a.kblock(from);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) a.Ak[base + i] = sk[i];
    if constexpr (VB != 0) {
        const auto* sv = a.vblock(from);
        for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) a.Av[base + i] = sv[i];
    }
}

// ---- F2: ordered compaction -----------------------------------------------------------

// gap[i] = sum of (b - len) over partial entries 0 .. i-1 of P; gap[sigma] = total
__global__ __launch_bounds__(256) void k_fin_gaps(const uint32_t* Pidx, const uint32_t* Plen,
                                                  uint32_t sigma, uint32_t log2b, uint32_t npi,
                                                  uint32_t* gap)
{
    extern __shared__ uint32_t s[];
    __shared__ uint32_t tmp[5];
    const uint32_t b = 1u << log2b;
    for (uint32_t i = threadIdx.x; i < sigma; i += 256) s[i] = Pidx[i] < npi ? b - Plen[i] : 0u;
    __syncthreads();
    uint32_t total = block_excl_scan<256>(s, sigma, tmp);
    for (uint32_t i = threadIdx.x; i < sigma; i += 256) gap[i] = s[i];
    if (threadIdx.x == 0) gap[sigma] = total;
}

// Unused elements before logical block L and the length of L.
__device__ __forceinline__ void gap_before(const uint32_t* Pidx, const uint32_t* Plen,
                                           const uint32_t* gap, uint32_t sigma, uint32_t L,
                                           uint32_t b, uint32_t& G, uint32_t& len)
{
    uint32_t lo = 0, hi = sigma;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (Pidx[mid] < L) lo = mid + 1;
        else hi = mid;
    }
    G = gap[lo];
    len = (lo < sigma && Pidx[lo] == L) ? Plen[lo] : b;
}

// One chunk = CHUNK consecutive element positions of the A blocks (whole blocks,
// or a part of one block when b > CHUNK), held in registers.  A chunk waits only
// for lower chunks to have loaded.  Persistent form (DYN = false): launched
// cooperatively, workgroup w takes chunks w, w + G, ...  Dynamic form: one
// workgroup per chunk, each claiming the next chunk from a counter (flags[chunks],
// zero on entry), so every lower chunk is held by a running workgroup.
template <int KB, int VB, int CHUNK, int NT, bool DYN = false>
__global__ __launch_bounds__(NT) void k_fin_compact(FinArgs<KB, VB> a, const uint32_t* gap,
                                                    uint32_t* flags, uint32_t chunks)
{
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    constexpr uint32_t MAXB = CHUNK / 64;
    constexpr int PER = CHUNK / NT;
    __shared__ uint32_t bG[MAXB], bL[MAXB];
    const uint32_t tid = threadIdx.x, b = 1u << a.log2b, sigma = a.sigma, log2b = a.log2b;
    const uint64_t total = (a.n >> log2b) << log2b;  // positions of the full A blocks
    const uint32_t fcur = *a.f;  // blocks at or past f hold no data (after truncate)
    uint32_t c0 = blockIdx.x, step = gridDim.x;
    if constexpr (DYN) {
        __shared__ uint32_t claimed;
        if (tid == 0) claimed = add_agent(flags + chunks, 1u);
        __syncthreads();
        c0 = claimed;
        step = chunks;
    }
    for (uint32_t c = c0; c < chunks; c += step) {
        __syncthreads();  // the previous chunk is done with bG / bL
        const uint64_t p0 = (uint64_t)c * CHUNK;
        const uint32_t cnt = (uint32_t)min<uint64_t>(CHUNK, total - p0);
        const uint64_t j0 = p0 >> log2b;
        const uint32_t nblk = (uint32_t)(((p0 + cnt - 1) >> log2b) - j0 + 1);
        for (uint32_t i = tid; i < nblk; i += NT) {
            uint32_t G, len;
            const uint32_t L = sigma + (uint32_t)(j0 + i);
            gap_before(a.Pidx, a.Plen, gap, sigma, L, b, G, len);
            bG[i] = G;
            bL[i] = L < fcur ? len : 0u;
        }
        __syncthreads();
        if (bG[nblk - 1] == 0) {  // no gap before this chunk: it stays where it is
            if (tid == 0) st_agent(flags + c, 1u);
            continue;
        }
        // load (elements beyond a block's length are never read)
        K rk[PER];
        V rv[PER];
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const uint32_t i = k * NT + tid;
            const uint64_t pos = p0 + i;
            const uint32_t jb = (uint32_t)((pos >> log2b) - j0), off = (uint32_t)pos & (b - 1);
            const bool v = i < cnt && off < bL[jb];
            rk[k] = v ? a.Ak[pos] : (K)0;
            if constexpr (VB != 0) rv[k] = v ? a.Av[pos] : (V)0;
        }
        __builtin_amdgcn_s_waitcnt(0);  // every load of this thread has returned
        __syncthreads();
        if (tid == 0) st_agent(flags + c, 1u);
        // wait for the chunks whose sources overlap the destination
        const uint64_t dst0 = p0 - bG[0];
        const uint32_t cfirst = (uint32_t)(dst0 / CHUNK);
        for (uint32_t w = cfirst + tid; w < c; w += NT) {
            uint32_t spins = 0;
            while (ld_agent(flags + w) == 0u) {
                if (spin_give_up(++spins, a.err)) break;
                spin_pause();
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const uint32_t i = k * NT + tid;
            const uint64_t pos = p0 + i;
            const uint32_t jb = (uint32_t)((pos >> log2b) - j0), off = (uint32_t)pos & (b - 1);
            if (i < cnt && off < bL[jb]) {
                if (bG[jb] > pos) {  // never for a consistent P
                    raise_error(a.err, kErrBounds);
                    continue;
                }
                const uint64_t dst = pos - bG[jb];
                a.Ak[dst] = rk[k];
                if constexpr (VB != 0) a.Av[dst] = rv[k];
            }
        }
    }
}

// ---- F3: blocks resident in T ------------------------------------------------------

template <int KB, int VB>
__global__ __launch_bounds__(256) void k_fin_tail(FinArgs<KB, VB> a, const uint32_t* gap)
{
    const uint32_t sigma = a.sigma, b = 1u << a.log2b, nb = (uint32_t)(a.n >> a.log2b);
    const uint32_t L = sigma + nb + blockIdx.x;
    if (L >= *a.f || L >= a.npi) return;
    uint32_t G, len;
    gap_before(a.Pidx, a.Plen, gap, sigma, L, b, G, len);
    const uint32_t phys = L + sigma - a.npi;  // rot(L) for L >= n_pi - sigma
    const uint64_t dst = ((uint64_t)(L - sigma) << a.log2b) - G;
    if (dst + len > a.n) {  // never for a consistent state
        raise_error(a.err, kErrBounds);
        return;
    }
    for (uint32_t i = threadIdx.x; i < len; i += 256) {
        a.Ak[dst + i] = a.Tk[((uint64_t)phys << a.log2b) + i];
        if constexpr (VB != 0) a.Av[dst + i] = a.Tv[((uint64_t)phys << a.log2b) + i];
    }
}

// ---- host launch sequence ----------------------------------------------------------

inline void fin_scan(uint32_t* a, uint32_t count, uint32_t* sums, hipStream_t s)
{
    const uint32_t tiles = (count + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(256), 0, s, a, count, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, tiles);
    hipLaunchKernelGGL(k_scan_add, dim3(tiles), dim3(256), 0, s, a, count, sums);
}

// F2's chunk and its persistent launch: compact_grid workgroups of kCompactThreads,
// at most as many as are resident at once (the caller gets it from the occupancy
// of k_fin_compact<KB, VB, fin_chunk<KB, VB>(), kCompactThreads>).
constexpr int kCompactThreads = 512;
template <int KB, int VB> constexpr int fin_chunk() { return (KB + VB >= 12) ? 4096 : 8192; }

// compact_grid = 0 selects the dynamic compaction (one workgroup per chunk);
// lds_grid = 0 the two-kernel F1 with heads saved in global memory, else the
// cooperative F1 on lds_grid workgroups (one per compute unit)
// temps: the scratch holds the two-kernel form's temporary blocks (fin_scratch_bytes);
// without them a state the cooperative form cannot cover returns -2 before any launch
template <int KB, int VB>
int finalize_parallel(FinArgs<KB, VB>& a, uint32_t compact_grid, uint32_t lds_grid,
                      bool temps, hipStream_t s)
{
    const FinCoop coop = fin_coop(a.npi, 1u << a.log2b, KB + VB, lds_grid);
    if (!coop.covers && !temps) return -2;
    const uint32_t npi = a.npi, b = 1u << a.log2b;
    FinArrays f = fin_arrays(a.scratch, npi, a.n, a.spare_pi, a.spare_blen);
    const uint32_t grid = std::min<uint32_t>((npi + 255) / 256, 8192);
    uint32_t* rank = f.j0;
    uint32_t* clen = f.j1;
    const uint32_t* M_ptr;  // total number of nodes to move
    uint32_t* gap;          // F2's gap prefix
    // a packed state: its bucket table, then every logical block's home (in o1,
    // which the preparation below reads before it writes o1)
    const uint32_t* homes = nullptr;
    if (a.pack) {
        hipLaunchKernelGGL(k_pack_table<256>, dim3(1), dim3(256), 8 * a.sigma, s, a.est, a.n,
                           a.sigma, a.log2b, a.pack);
        hipLaunchKernelGGL(k_pack_homes, dim3(grid), dim3(256), 0, s, a.S, a.est, a.f, a.pack,
                           a.n, a.sigma, a.log2b, a.npi_eq, npi, f.o1, a.err);
        homes = f.o1;
    }
    const bool small = npi <= kFinSmallNodes;
    if (small) {
        // F1's preparation, F2's gaps and flags in one workgroup
        hipLaunchKernelGGL(k_fin_prep_small<1024>, dim3(1), dim3(1024), 0, s, a.pi, a.f, a.Pidx,
                           a.Plen, a.sigma, a.log2b, npi, rank, clen, f.ord, f.sums, f.o0,
                           f.flags, f.nflags, a.err, homes);
        M_ptr = f.sums;
        gap = f.o0;
    } else {
        // F1: cycles
        uint32_t *J[2] = {f.j0, f.j1}, *Vv[2] = {f.v0, f.v1}, *O[2] = {f.o0, f.o1};
        hipLaunchKernelGGL(k_fin_init, dim3(grid), dim3(256), 0, s, a.pi, a.f, a.sigma, npi,
                           f.nxt, J[0], Vv[0], O[0], homes);
        // windows of 4^k successors: ceil(log4 n_pi) launches
        int cur = 0;
        for (uint64_t w = 1; w < npi; w <<= 2) {
            hipLaunchKernelGGL(k_fin_jump4, dim3(grid), dim3(256), 0, s, J[cur], Vv[cur], O[cur],
                               J[cur ^ 1], Vv[cur ^ 1], O[cur ^ 1], npi, (uint32_t)w);
            cur ^= 1;
        }
        uint32_t* V = Vv[cur];
        uint32_t* Ofin = O[cur];
        uint32_t* scan = Vv[cur ^ 1];
        hipLaunchKernelGGL(k_fin_rank, dim3(grid), dim3(256), 0, s, f.nxt, V, Ofin, rank, clen,
                           scan, npi);
        fin_scan(scan, npi, f.sums, s);
        const uint32_t tiles = (npi + kScanTile - 1) / kScanTile;
        M_ptr = f.sums + tiles;
        hipLaunchKernelGGL(k_fin_order, dim3(grid), dim3(256), 0, s, f.nxt, V, rank, clen, scan,
                           f.ord, npi);
        // F2's gap prefix goes where the doubling state was (free after k_fin_order);
        // a packed state has no F2
        gap = Ofin;
        if (!a.pack) {
            hipLaunchKernelGGL(k_fin_gaps, dim3(1), dim3(256), 4 * a.sigma, s, a.Pidx, a.Plen,
                               a.sigma, a.log2b, npi, gap);
            hipLaunchKernelGGL(k_fill_u32,
                               dim3((uint32_t)std::min<uint64_t>((f.nflags + 255) / 256, 4096)),
                               dim3(256), 0, s, f.flags, f.nflags, 0u);
        }
    }
    // four columns per thread when every block start is 16-byte aligned
    const bool wide = b >= 64 && (((uintptr_t)a.Ak | (uintptr_t)a.Av | (uintptr_t)a.Tk |
                                   (uintptr_t)a.Tv | (uintptr_t)f.temps) & 15) == 0;
    const uint64_t head_bytes = (uint64_t)b * (KB + VB);
    // the cooperative form when it covers every node, else the two-kernel form
    if (coop.covers) {
        uint32_t job = coop.job, jpw = coop.jpw;
        const uint32_t grid = coop.grid;
        const uint32_t lds = (uint32_t)(2 * jpw * head_bytes);
        void* args[] = {(void*)&a, (void*)&f, (void*)&rank, (void*)&clen, (void*)&M_ptr,
                        (void*)&job, (void*)&jpw};
        const void* kern = wide ? (const void*)&k_fin_move_lds<KB, VB, 4>
                                : (const void*)&k_fin_move_lds<KB, VB, 1>;
        if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
            return -1;
        if (hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kFinLdsThreads), args, lds, s) !=
            hipSuccess)
            return -1;
    } else {
    const uint32_t jobs = (npi + a.job - 1) / a.job;
    hipLaunchKernelGGL((k_fin_save<KB, VB>), dim3(jobs), dim3(256), 0, s, a, f, rank, clen, M_ptr);
    if (wide) {
        const uint32_t slices = (b + 4 * kFinCols - 1) / (4 * kFinCols);
        hipLaunchKernelGGL((k_fin_move<KB, VB, 4>), dim3(jobs, slices), dim3(kFinCols), 0, s, a, f,
                           rank, clen, M_ptr);
    } else {
        const uint32_t slices = (b + kFinCols - 1) / kFinCols;
        hipLaunchKernelGGL((k_fin_move<KB, VB, 1>), dim3(jobs, slices), dim3(kFinCols), 0, s, a, f,
                           rank, clen, M_ptr);
    }
    }
    // a packed state has no gaps to close: its blocks that do not end in A go in now
    if (a.pack) {
        hipLaunchKernelGGL((k_pack_merge<KB, VB>), dim3(a.sigma), dim3(256), 0, s, a);
        return 0;
    }
    // F2: compaction
    const uint64_t positions = (a.n >> a.log2b) << a.log2b;
    constexpr int CHUNK = fin_chunk<KB, VB>();
    uint32_t chunks = (uint32_t)((positions + CHUNK - 1) / CHUNK);
    if (chunks && compact_grid == 0) {
        hipLaunchKernelGGL((k_fin_compact<KB, VB, CHUNK, kCompactThreads, true>), dim3(chunks),
                           dim3(kCompactThreads), 0, s, a, gap, f.flags, chunks);
    } else if (chunks) {
        const uint32_t grid = std::min(chunks, compact_grid);
        void* args[] = {(void*)&a, (void*)&gap, (void*)&f.flags, (void*)&chunks};
        if (hipLaunchCooperativeKernel((const void*)&k_fin_compact<KB, VB, CHUNK, kCompactThreads>,
                                       dim3(grid), dim3(kCompactThreads), args, 0, s) != hipSuccess)
            return -1;
    }
    // F3: the blocks in T
    hipLaunchKernelGGL((k_fin_tail<KB, VB>), dim3(a.sigma), dim3(256), 0, s, a, gap);
    return 0;
}

}  // namespace rs
