// State kernels of Radsort: fills, the digit histograms of all key positions,
// the plan of a round (closed forms of C, S, P, f), setup (Alg. 4), fixupPhase
// (Alg. 6), truncate (Alg. 8) and the block table.
#pragma once

#include "common.hpp"

namespace rs {

__global__ void k_fill_u32(uint32_t* p, uint64_t count, uint32_t v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// A plain streaming copy of 16-byte words (the practical HBM ceiling the sort is
// measured against): every thread moves 4 words per step, all 4 loads issued
// before the stores, grid-stride over the buffer.  The bytes that do not fill a
// 16-byte word are copied by the first threads one byte each.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(u32x4* __restrict__ dst,
                                                     const u32x4* __restrict__ src,
                                                     uint64_t words, uint8_t* __restrict__ dtail,
                                                     const uint8_t* __restrict__ stail,
                                                     uint32_t tail)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < words; i += 4 * stride) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; u++) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < words; i += stride) dst[i] = src[i];
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < tail) dtail[t] = stail[t];
}

// Histograms of every key position in one pass over the keys (the first loop
// of Alg. 1, taken for all positions up front as the paper's "generic" variant
// does, Sec. 5).  hist[t * sigma + c] counts key(x, t) = c, t = 0 the most
// significant digit.  hist must be zero on entry.  Dynamic LDS: copies * nt *
// sigma words, copies = the number of waves sharing a copy of the counts (each
// wave adds into copy wave % copies).
template <int KB, int NT>
__global__ __launch_bounds__(NT) void k_histograms(const typename UInt<KB>::T* __restrict__ keys,
                                                   uint64_t n, uint32_t bits, uint32_t nt,
                                                   uint32_t copies, uint32_t* __restrict__ hist)
{
    using K = typename UInt<KB>::T;
    constexpr int U = 8;  // loads in flight per thread
    extern __shared__ uint32_t h[];
    const uint32_t sigma = 1u << bits, mask = sigma - 1, words = nt * sigma;
    for (uint32_t i = threadIdx.x; i < copies * words; i += NT) h[i] = 0;
    __syncthreads();
    uint32_t* mine = h + ((threadIdx.x >> 6) % copies) * words;
    const uint64_t step = (uint64_t)gridDim.x * NT * U;
    for (uint64_t c = (uint64_t)blockIdx.x * NT * U; c < n; c += step) {
        K x[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const uint64_t i = c + (uint64_t)j * NT + threadIdx.x;
            x[j] = i < n ? keys[i] : (K)0;
        }
#pragma unroll
        for (int j = 0; j < U; j++) {
            if (c + (uint64_t)j * NT + threadIdx.x < n) {
                for (uint32_t t = 0; t < nt; t++) {
                    const uint32_t d = (uint32_t)(x[j] >> (bits * (nt - 1 - t))) & mask;
                    atomicAdd(&mine[t * sigma + d], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < words; i += NT) {
        uint32_t v = 0;
        for (uint32_t k = 0; k < copies; k++) v += h[k * words + i];
        if (v) atomicAdd(&hist[i], v);
    }
}

// Everything a round needs that follows from the digit counts of its input alone,
// by the closed forms of Alg. 5 (eager allocation) and Alg. 6:
//   C[d]   = 1 + floor(cnt_d / b)                     blocks of bucket d
//   S[d]   = sigma + sum_{d' < d} C[d']               first logical block of d
//   P[d]   = (S[d] + C[d] - 1, cnt_d mod b)           its partial block
//   f      = sigma + sum_d C[d]
//   est[d] = sum_{d' < d} cnt_d'                      element start (Alg. 1)
// Round r sorts by key position t = nt-1-r.  P and f of index r describe the
// input of round r; index 0 is the state after setup (Alg. 4).
struct PlanPtrs {
    uint32_t* S;     // [nt][sigma]
    uint32_t* Pidx;  // [nt+1][sigma]
    uint32_t* Plen;  // [nt+1][sigma]
    uint32_t* f;     // [nt+1]
    uint32_t* est;   // [nt][sigma]
};

// One round of the plan from the digit counts cnt[0..sigma) of its input.  C and
// E are sigma words of LDS each, tmp NT/64 + 1; est may be null (Radsort itself
// needs no element starts).  Contains barriers: every thread must call it.
//
// packed (a Radsort round that is the last before finalize; est given): bucket d
// starts at offset o_d = est[d] mod b of its head block, so that its ranks sit at
// the slots their final positions est[d] + rank have within blocks of A.  Its
// blocks are those of o_d + c_d ranks: C[d] = 1 + floor((o_d + c_d) / b), the last
// one partial with (o_d + c_d) mod b slots up to its end; the first one holds
// slots o_d .. b - 1 only.
template <int NT>
__device__ void plan_round(const uint32_t* __restrict__ cnt, uint32_t sigma, uint32_t log2b,
                           uint32_t* C, uint32_t* E, uint32_t* tmp, uint32_t* __restrict__ S,
                           uint32_t* __restrict__ Pidx, uint32_t* __restrict__ Plen,
                           uint32_t* __restrict__ f, uint32_t* __restrict__ est,
                           bool packed = false)
{
    const uint32_t b = 1u << log2b, tid = threadIdx.x;
    for (uint32_t d = tid; d < sigma; d += NT) E[d] = cnt[d];
    __syncthreads();
    if (est) block_excl_scan<NT>(E, sigma, tmp);
    // ranks of bucket d as the blocks see them: its count, plus o_d when packed
    auto span = [&](uint32_t d) { return cnt[d] + (packed ? (E[d] & (b - 1)) : 0u); };
    for (uint32_t d = tid; d < sigma; d += NT) C[d] = 1 + (span(d) >> log2b);
    __syncthreads();
    const uint32_t total = block_excl_scan<NT>(C, sigma, tmp);
    for (uint32_t d = tid; d < sigma; d += NT) {
        const uint32_t c = 1 + (span(d) >> log2b);
        const uint32_t s = sigma + C[d];
        S[d] = s;
        Pidx[d] = s + c - 1;
        Plen[d] = span(d) & (b - 1);
        if (est) est[d] = E[d];
    }
    if (tid == 0) *f = sigma + total;
    __syncthreads();
}

// setup (Alg. 4): pi = [0..sigma) | 2 sigma .. sigma + f - 2 | sigma .. 2 sigma),
// the n mod b tail of A copied to physical block sigma, the other pi buffer
// cleared to "unset", f = sigma + floor(n/b) + 1 and P = the tail block, then
// dummies (Pidx, Plen, f_out: index 0 of the per-round arrays); the first
// round's look-back ring (ring_words words) cleared.
template <int KB, int VB>
__global__ void k_setup(typename UInt<KB>::T* __restrict__ Ak,
                        typename Payload<VB>::T* __restrict__ Av,
                        typename UInt<KB>::T* __restrict__ Tk,
                        typename Payload<VB>::T* __restrict__ Tv, uint64_t n, uint32_t log2b,
                        uint32_t sigma, uint32_t npi, uint32_t* __restrict__ pi,
                        uint32_t* __restrict__ pi_next, uint32_t* __restrict__ blen,
                        uint64_t* __restrict__ opened, uint32_t* __restrict__ Pidx,
                        uint32_t* __restrict__ Plen, uint32_t* __restrict__ f_out,
                        uint32_t* __restrict__ ring, uint64_t ring_words)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < ring_words;
         i += (uint64_t)gridDim.x * blockDim.x)
        ring[i] = 0;
    const uint64_t nb = n >> log2b, tail = n - (nb << log2b);
    const uint32_t f = sigma + (uint32_t)nb + 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < npi || i < tail;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (i < sigma) {
            Pidx[i] = i == 0 ? f - 1 : npi;  // the input tail, then dummies
            Plen[i] = i == 0 ? (uint32_t)tail : 0u;
            if (i == 0) *f_out = f;
        }
        if (i < npi) {
            uint32_t L = (uint32_t)i, v;
            if (L < sigma) v = L;
            else if (L + 1 < f) v = L + sigma;
            else v = sigma + (L - (f - 1));
            pi[L] = v;
            pi_next[L] = kEmpty;
            // used lengths: full blocks, and the tail as logical f - 1 (Alg. 4)
            blen[L] = L + 1 == f ? (uint32_t)tail : (1u << log2b);
            if (L < sigma) opened[L] = 0;
        }
        if (i < tail) {
            uint64_t dst = ((uint64_t)sigma << log2b) + i;
            Tk[dst] = Ak[(nb << log2b) + i];
            if constexpr (VB != 0) Tv[dst] = Av[(nb << log2b) + i];
        }
    }
}

// fixupPhase (Alg. 6) after a sort round.  The sort round already wrote
// pi_new[S[d] + q] for every block q >= 1 of every bucket (the blocks drawn when
// a block filled).  Here: the first block of bucket d is pool entry d (the
// initial newBucketBlock draws of Alg. 5), the head start is pool entries
// c .. c + sigma - 1 and the rest keeps its place, with c = f_out - sigma the
// number of blocks drawn.  Each entry of pi_old is read by the thread that owns
// it, which then resets it to "unset" for the next round.
// It also writes the used length of every logical block for the next round:
// b, or the length recorded in P for the buckets' last blocks, and clears the
// next round's look-back ring (ring_words words).
__global__ void k_fixup(uint32_t* __restrict__ pi_old, uint32_t* __restrict__ pi_new,
                        const uint32_t* __restrict__ S, const uint32_t* __restrict__ f_out,
                        const uint32_t* __restrict__ Pidx, const uint32_t* __restrict__ Plen,
                        uint32_t* __restrict__ blen, uint64_t* __restrict__ opened,
                        uint32_t sigma, uint32_t log2b, uint32_t npi, uint32_t* __restrict__ ring,
                        uint64_t ring_words)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < ring_words;
         i += (uint64_t)gridDim.x * blockDim.x)
        ring[i] = 0;
    const uint32_t c = *f_out - sigma;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < npi;
         j += gridDim.x * blockDim.x) {
        if (j < sigma) opened[j] = 0;  // per-bucket latest draw, for the next round
        uint32_t v = pi_old[j];
        if (j < sigma) {
            if (S[j] < npi) pi_new[S[j]] = v;
        }
        else if (j >= c && j < c + sigma) pi_new[j - c] = v;
        else if (j >= c + sigma) pi_new[j] = v;
        pi_old[j] = kEmpty;
        uint32_t lo = 0, hi = sigma;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (Pidx[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        blen[j] = (lo < sigma && Pidx[lo] == j) ? Plen[lo] : (1u << log2b);
    }
}

// After a packed round (plan_round): pi' over all npi + sigma logical blocks, as
// k_fixup builds it.  The buckets' first blocks are their head blocks (logical
// 0 .. sigma - 1 of the round's input); the round drew the first f - 2 sigma
// entries of its pool (the sigma extra blocks npi .., then pi[sigma ..]); the
// entries it left fill logical blocks 0 .. sigma - 1 and f .. npi + sigma - 1.
__global__ void k_pack_fixup(const uint32_t* __restrict__ pi_old, uint32_t* __restrict__ pi_new,
                             const uint32_t* __restrict__ S, const uint32_t* __restrict__ f_out,
                             uint32_t sigma, uint32_t npi)
{
    const uint32_t npx = npi + sigma, f = min(max(*f_out, 2 * sigma), npx);
    const uint32_t drawn = f - 2 * sigma;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < npx;
         j += gridDim.x * blockDim.x) {
        if (j < sigma) {
            if (S[j] < npx) pi_new[S[j]] = pi_old[j];
            const uint32_t k = drawn + j;  // < npi, as f <= npi + sigma
            pi_new[j] = k < sigma ? npi + k : pi_old[k];
        } else if (j >= f) {
            pi_new[j] = pi_old[j - sigma];
        }
    }
}

// ---- the permuted representation without finalize (Sec. 4.1) -------------------

__global__ void k_copy_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                           uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// truncate (Alg. 8) to the first `count` elements of the logical sequence, on the
// state (P, f, block lengths) of the current round.  One workgroup.
// The block holding element q = count - 1 is found from P: every block between
// two partial blocks is full, so with E_e = the elements before partial block
// Pidx[e] ((Pidx[e] - sigma) b minus the unused room of the partial blocks
// before it), q lies in the first partial block that ends after it or in one of
// the full blocks just before that block.  With (i, j) its block and offset, f
// becomes i + 1 and that entry of P becomes (i, j + 1) (Alg. 8); the entries
// after it name blocks past the new f and are left alone.  count = 0 gives
// (sigma, 0): an empty dataset.  Entries at or past f (left by an earlier
// truncate) and the dummies of setup take no part.  Dynamic LDS: sigma words.
template <int NT>
__global__ __launch_bounds__(NT) void k_truncate(uint32_t* __restrict__ Pidx,
                                                 uint32_t* __restrict__ Plen,
                                                 uint32_t* __restrict__ f_ptr,
                                                 uint32_t* __restrict__ blen, uint32_t sigma,
                                                 uint32_t log2b, uint64_t count,
                                                 uint32_t* __restrict__ err)
{
    extern __shared__ uint32_t gap[];
    __shared__ uint32_t tmp[NT / 64 + 1];
    __shared__ uint32_t found, fe, fi, fj;
    const uint32_t tid = threadIdx.x, b = 1u << log2b, f = *f_ptr;
    if (tid == 0) found = 0;
    for (uint32_t e = tid; e < sigma; e += NT) gap[e] = Pidx[e] < f ? b - min(Plen[e], b) : 0u;
    __syncthreads();
    block_excl_scan<NT>(gap, sigma, tmp);  // gap[e] = unused room before block Pidx[e]
    if (count == 0) {
        if (tid == 0) {
            fe = 0;
            fi = sigma;
            fj = 0;
            found = 1;
        }
    } else {
        const uint64_t q = count - 1;
        for (uint32_t e = tid; e < sigma; e += NT) {
            const uint32_t idx = Pidx[e];
            if (idx >= f) continue;
            const uint64_t before = ((uint64_t)(idx - sigma) << log2b) - gap[e];
            const uint64_t end = before + min(Plen[e], b);
            // elements through the previous partial block, and the block after it
            uint64_t prev_end = 0;
            uint32_t first = sigma;
            if (e > 0) {
                const uint32_t pidx = Pidx[e - 1];
                prev_end = ((uint64_t)(pidx - sigma) << log2b) - gap[e - 1] + min(Plen[e - 1], b);
                first = pidx + 1;
            }
            if (end <= q || (e > 0 && prev_end > q)) continue;  // not the first to pass q
            fe = e;  // exactly one entry passes
            if (q >= before) {
                fi = idx;
                fj = (uint32_t)(q - before) + 1;
            } else {  // a full block between the two partial blocks
                fi = first + (uint32_t)((q - prev_end) >> log2b);
                fj = (uint32_t)((q - prev_end) & (b - 1)) + 1;
            }
            found = 1;
        }
    }
    __syncthreads();  // every read of P is done before the writes
    if (tid == 0) {
        if (!found) {  // count past the data: the state is left as it is
            raise_error(err, kErrBounds);
        } else {
            Pidx[fe] = fi;
            Plen[fe] = fj;
            *f_ptr = fi + 1;
            blen[fi] = fj;
        }
    }
}

// The block table of the permuted representation: for logical block L = sigma ..
// n_pi - 1, phys[L - sigma] = pi[L] and len[L - sigma] = its used length, or
// (0xFFFFFFFF, 0) for the unallocated blocks L >= f.
__global__ void k_block_table(const uint32_t* __restrict__ pi, const uint32_t* __restrict__ blen,
                              const uint32_t* __restrict__ f_ptr, uint32_t sigma, uint32_t npi,
                              uint32_t log2b, uint32_t* __restrict__ phys,
                              uint32_t* __restrict__ len)
{
    const uint32_t f = *f_ptr;
    for (uint32_t L = sigma + blockIdx.x * blockDim.x + threadIdx.x; L < npi;
         L += gridDim.x * blockDim.x) {
        const bool used = L < f;
        if (phys) phys[L - sigma] = used ? pi[L] : 0xFFFFFFFFu;
        if (len) len[L - sigma] = used ? min(blen[L], 1u << log2b) : 0u;
    }
}

}  // namespace rs
