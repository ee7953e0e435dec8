/*
 * radsort.h -- C ABI of the MI355X (gfx950) Radsort library.
 *
 * Radsort is the stable LSD radix sort with O(sqrt n) extra space of
 * "Parallel O(sqrt n) Overhead LSD Radix Sort" (Clausecker, Schintke).  The
 * problem statement (Sec. 1) is: sort an array A of n elements whose keys are
 * n_t-tuples of digits over an alphabet of sigma symbols into lexicographic
 * order by stable rounds on key positions n_t-1, ..., 0.  Here keys are unsigned
 * integers of key_bytes bytes split into digits of digit_bits bits, so sigma =
 * 2^digit_bits and n_t = ceil(8 key_bytes / digit_bits); position n_t-1 is the
 * least significant digit.  The result is ascending by unsigned key and stable.
 *
 * Conventions for every call:
 *   - keys and payload are DEVICE pointers to n contiguous elements each
 *     (structure of arrays; the two ranges must not overlap).  They stay owned by
 *     the caller.  Their contents are undefined from the call until the stream
 *     reaches the end of the work the call enqueued.
 *   - stream is a hipStream_t (NULL = the null stream).  Work is enqueued on it;
 *     unless stated otherwise a call returns without waiting for the GPU.
 *   - workspace: device memory of at least the queried size, owned by the caller,
 *     untouched by anyone else until the enqueued work has finished.  When
 *     opts->workspace is NULL the library allocates the workspace itself for the
 *     call and waits for the stream before freeing it.
 *   - return value: RADSORT_OK (0) or a negative RADSORT_E_* code.  Argument
 *     errors are detected before anything is enqueued and leave the data as it
 *     was.  After a device error the data is undefined.
 *   - digit_bits is 1 .. 16 as an argument (sigma up to 2^16); widths 12 .. 16
 *     return RADSORT_E_UNSUPPORTED from every call.  Three costs rule them out
 *     on this GPU: (1) the 2 sigma head blocks of the state (Sec. 2.1) hold
 *     2 sigma b elements, which stays within 1 % of n only for n >= 200 sigma b
 *     (at 16 bits and b = 1024: 1.3e10 elements, above the 2^32 limit);
 *     (2) a tile's per-wave digit counts take waves * sigma * 4 bytes of LDS
 *     (at 16 bits: 1 MiB for 4 waves, beyond the 160 KiB of a compute unit);
 *     (3) a tile holds 2048 to 8192 elements, so with sigma >= 2^12 a digit's
 *     run in a tile averages two elements or fewer and the scatter writes
 *     mostly partial 128-byte lines, costing more bytes than the round that the
 *     wider digit saves (32-bit keys: 3 rounds at 11 bits, 2 at 16).
 */
#ifndef RADSORT_H
#define RADSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RADSORT_OK 0
#define RADSORT_E_INVALID (-1)      /* bad argument: null pointer with n > 0, widths, b */
#define RADSORT_E_NOMEM (-2)        /* allocation failed or workspace too small */
#define RADSORT_E_DEVICE (-3)       /* a HIP call failed; see radsort_strerror */
#define RADSORT_E_UNSUPPORTED (-4)  /* n >= 2^32 or digit_bits 12 .. 16 */
#define RADSORT_E_TIMEOUT (-5)      /* a device-side check failed: a bounded wait gave
                                       up, or an index left its range */
#define RADSORT_E_ORDER (-6)        /* RADSORT_F_DEBUG_ORDER: a block was drawn before the
                                       loads of its readers were marked returned */

/* flags of radsort_opts */
#define RADSORT_F_CHECK 1u          /* wait for the stream and report device-side errors */
#define RADSORT_F_TIMING 2u         /* record HIP events around each phase on the stream;
                                       radsort_last_stats() waits for them and reports */
#define RADSORT_F_SHARED 4u         /* the GPU runs other work at the same time: use launch
                                       forms that need no co-resident grid (one workgroup
                                       per tile, tiles claimed in order).  Those forms are
                                       taken anyway, being faster, by radsort_sort_pairs
                                       with block_elems <= 1024 and always by
                                       radsort_oop_sort_pairs */
#define RADSORT_F_SEQ_DRAWS 8u      /* Radsort rounds draw their blocks in the order of the
                                       sequential scan of Alg. 5 (the elements that fill
                                       the blocks, in input order), so that pi after every
                                       round equals the sequential algorithm's.  Without it
                                       the draws of one tile go in (digit, block) order:
                                       the same pool entries per tile (Lemma 1 holds alike),
                                       the same P, f and logical contents, a different pi;
                                       faster.  Digits of more than 8 bits always draw in
                                       the sequential order */

#define RADSORT_F_DEBUG_ORDER 16u   /* ordering check (the library built with RS_DEBUG_ORDER
                                       defined; any other build returns
                                       RADSORT_E_UNSUPPORTED): every Radsort round marks
                                       each input block once the loads of the tile that
                                       reads it have returned, and every draw of a block
                                       holding input of the round checks the mark; a
                                       missing mark sets error bit 4 (radsort_stats) and
                                       the call returns RADSORT_E_ORDER.  Needs b <= the
                                       round's tile (8192 elements for 4-byte keys);
                                       slower; for tests.  With RADSORT_F_DEBUG_PLANT as
                                       well the marks carry a wrong tag, so that every
                                       checked draw reports (a test of the check) */
#define RADSORT_F_DEBUG_PLANT 0x80000000u

typedef struct radsort_opts {
    uint32_t block_elems;     /* b: block size in elements, a power of two in [64, 65536];
                                 0 selects 1024 */
    uint32_t tile_elems;      /* reserved, 0 */
    void* workspace;          /* device workspace, or NULL: allocated per call */
    uint64_t workspace_bytes; /* its size in bytes */
    uint32_t flags;           /* RADSORT_F_* */
} radsort_opts;

#define RADSORT_MAX_ROUNDS 64

/* Block size and digit width per size class for the arrays of radsort_sort_segments
 * that run the Radsort steps on streams: an array of n elements takes the first class
 * c with ceil(log2 n) <= max_log2n[c].  Arrays above 4 423 680 elements always run
 * there; a smaller array (but above the whole-in-LDS limit of 8192, or 4096 for
 * records of 12 bytes or more) runs there when its class has block_elems > 0, and on
 * one workgroup of the batched kernel when block_elems = 0 or no class covers it.
 * digit_bits must be 4, 8 or 11 and block_elems 0 or a power of two in [64, 65536];
 * a class with block_elems = 0 takes the batched kernel's own digits (5 bits, b =
 * 1024) and its digit_bits is not used. */
#define RADSORT_SEG_CLASSES 32
typedef struct radsort_seg_tuning {
    uint32_t classes;
    uint32_t max_log2n[RADSORT_SEG_CLASSES];
    uint32_t block_elems[RADSORT_SEG_CLASSES];
    uint32_t digit_bits[RADSORT_SEG_CLASSES];
} radsort_seg_tuning;

typedef struct radsort_stats {
    uint64_t workspace_bytes;   /* extra device bytes of the last sort (peak extra memory) */
    uint64_t input_bytes;       /* n * (key_bytes + payload_bytes) of the last sort */
    uint32_t rounds;            /* digit rounds run */
    uint32_t error_bits;        /* device error word of the last checked call */
    /* with RADSORT_F_TIMING: milliseconds between HIP events on the call's stream */
    uint32_t timed;             /* 1 when the fields below are valid */
    float setup_ms;             /* setup (Alg. 4) */
    float round_ms[RADSORT_MAX_ROUNDS]; /* the sort-round kernel of each round (Alg. 5) */
    float count_ms[RADSORT_MAX_ROUNDS]; /* each round's super-tile digit counts, their scan
                                           and the round's plan */
    float fixup_ms;             /* all fixup kernels (Alg. 6) and counter resets */
    float finalize_ms;          /* finalize (Alg. 7); for the baseline: a final copy-back */
    float total_ms;             /* first event to last event */
} radsort_stats;

/*
 * radsort_sort_pairs -- sort keys[0..n) in place, ascending and stable, moving
 * payload[i] with keys[i].  Radsort, the driver of Alg. 2: setup (Alg. 4), then
 * for t = n_t-1 .. 0 a sort phase (Alg. 5) and a fixup phase (Alg. 6), then
 * finalize (Alg. 7).  Each round first counts the digits of its own input (the
 * histogram loop of Alg. 1, per group of tiles) and takes its bucket starts and
 * the P and f it leaves from those counts by closed forms.  The last round is
 * packed (see radsort_workspace_bytes): every element lands at the slot of its
 * final position, so that finalize permutes whole blocks and merges at most one
 * partial block per bucket, with no compaction; the result is the same.
 *   key_bytes      4 or 8 (uint32 / uint64 keys; signed or float keys are not
 *                  handled: the order is that of the unsigned bit patterns)
 *   payload_bytes  0 (payload must be NULL), 4 or 8
 *   digit_bits     1 .. 11 (12 .. 16: RADSORT_E_UNSUPPORTED; 0 or > 16: INVALID)
 *   opts           may be NULL (b = 1024, library-allocated workspace)
 * Extra device memory is the workspace only: radsort_workspace_bytes().
 * n <= 1 returns RADSORT_OK without touching the data.
 */
int radsort_sort_pairs(void* keys, void* payload, uint64_t n, int key_bytes,
                       int payload_bytes, int digit_bits, const radsort_opts* opts,
                       void* stream);

/*
 * radsort_workspace_error -- the device-side error word that the last
 * radsort_sort_pairs (out_of_place = 0) or radsort_oop_sort_pairs (out_of_place = 1)
 * call with this workspace left, for callers that pass their own workspace and no
 * RADSORT_F_CHECK, so that the sort itself returned without waiting.  n, key_bytes,
 * payload_bytes, digit_bits and opts (workspace, workspace_bytes, block_elems) must
 * be those of that call.  Enqueues a 4-byte copy on `stream` and waits for the
 * stream.  *error_bits (may be NULL) receives the word: 0, or bit 0 when a bounded
 * wait between workgroups gave up, bit 1 when an index fell outside its array (the
 * data are then unspecified).  Returns RADSORT_OK for 0, RADSORT_E_TIMEOUT for any
 * bit, RADSORT_E_INVALID / RADSORT_E_NOMEM for a missing or short workspace.
 */
int radsort_workspace_error(const void* workspace, uint64_t n, int key_bytes,
                            int payload_bytes, int digit_bits, const radsort_opts* opts,
                            int out_of_place, uint32_t* error_bits, void* stream);

/* radsort_sort -- radsort_sort_pairs without payload and with default options. */
int radsort_sort(void* keys, uint64_t n, int key_bytes, int digit_bits, void* stream);

/* Workspace bytes radsort_sort_pairs needs for these arguments: the scratch
 * blocks T (2 sigma b elements, Sec. 2.1), two n_pi-entry block permutations,
 * the per-round closed forms, the digit counts and look-back status ring and the
 * finalize scratch (which reuses the ring's memory).  The size depends on
 * opts->flags and on the current device's compute-unit count (256 assumed when no
 * device answers), which decides whether the cooperative form of finalize's block
 * permutation covers the state.  Without RADSORT_F_SHARED, when it does, the last
 * round is packed: each bucket starts at the offset its final position has within
 * a block, so that finalize only permutes blocks (no compaction), which takes
 * sigma more blocks of b elements and n_pi + sigma entries per permutation.  With
 * RADSORT_F_SHARED the finalize scratch instead holds two blocks per job of the
 * permutation's two-kernel form.  0 on invalid arguments. */
uint64_t radsort_workspace_bytes(uint64_t n, int key_bytes, int payload_bytes,
                                 int digit_bits, const radsort_opts* opts);

/*
 * radsort_oop_sort_pairs -- the out-of-place LSD radix sort of Alg. 1 on the
 * same tile code: n_t rounds, each a stable counting sort from one array into a
 * second one of n elements, ping-ponging between the caller's arrays and
 * workspace buffers.  Same arguments, result and ownership as
 * radsort_sort_pairs; it needs n (key_bytes + payload_bytes) extra bytes plus the
 * digit count and look-back state: radsort_oop_workspace_bytes().
 */
int radsort_oop_sort_pairs(void* keys, void* payload, uint64_t n, int key_bytes,
                           int payload_bytes, int digit_bits, const radsort_opts* opts,
                           void* stream);
uint64_t radsort_oop_workspace_bytes(uint64_t n, int key_bytes, int payload_bytes,
                                     int digit_bits, const radsort_opts* opts);

/*
 * radsort_sort_segments -- sort nseg independent arrays in place, each stable and
 * ascending by unsigned key with its payload, in one call on one stream.  Array i
 * is elements [offsets[i], offsets[i+1]) of the key plane (and of the payload
 * plane).  Arrays of at most 8192 elements (4096 for records of 12 or more bytes)
 * are each sorted whole in LDS by one workgroup, with 8-bit digits and no
 * workspace.  Arrays of up to 4 423 680 elements are sorted by Radsort (Alg. 2:
 * setup, n_t x sortPhase + fixupPhase, finalize) run by one workgroup per array,
 * all of them in one launch, with 5-bit digits and b = 1024 (each of at most 256
 * workgroups owns a T of 2 * 32 * 1024 elements in the workspace).  Larger arrays
 * each run the Radsort steps with the block size and digit width of their size
 * class in `tuning` (NULL: b = 2^ceil(log2 sqrt n) in [64, 2048] and 8-bit digits,
 * after the b in Theta(sqrt n) of Sec. 3), in launch forms that need no
 * co-residency, spread over four streams forked from `stream` and joined back to
 * it.
 *   offsets      host array of nseg + 1 non-decreasing element offsets
 *   offsets_dev  the same array in device memory (read by the kernels; it must hold
 *                the same values)
 *   opts         block_elems is ignored; workspace / workspace_bytes as for
 *                radsort_sort_pairs (radsort_segments_workspace_bytes gives the
 *                size; with a caller workspace nothing is allocated, so the call can
 *                be captured into a HIP graph); flags: RADSORT_F_CHECK waits and
 *                reports device errors
 * Returns RADSORT_E_INVALID for a null or decreasing offsets array or bad widths,
 * and the errors of radsort_sort_pairs otherwise.
 */
int radsort_sort_segments(void* keys, void* payload, const uint64_t* offsets,
                          const uint64_t* offsets_dev, uint32_t nseg, int key_bytes,
                          int payload_bytes, const radsort_seg_tuning* tuning,
                          const radsort_opts* opts, void* stream);
/* Workspace of radsort_sort_segments for these arrays, or 0 on a bad argument. */
uint64_t radsort_segments_workspace_bytes(const uint64_t* offsets, uint32_t nseg, int key_bytes,
                                          int payload_bytes, const radsort_seg_tuning* tuning,
                                          const radsort_opts* opts);

/*
 * radsort_histograms -- the digit histograms of all key positions in one pass
 * over the keys: counts[t * sigma + c]
 * = number of i with key(keys[i], t) = c, t = 0 the most significant position
 * (the first loop of Alg. 1 for every position).  counts is a device array of
 * n_t * sigma uint32 that the call overwrites.
 */
int radsort_histograms(const void* keys, uint64_t n, int key_bytes, int digit_bits,
                       uint32_t* counts, void* stream);

/* Statistics of the last sort call made by the calling host thread (each thread
 * keeps its own record; calls that one thread makes on several streams overwrite
 * it, and each call's device-side error word stays readable per workspace through
 * radsort_workspace_error).  If that call asked for RADSORT_F_TIMING, this waits
 * for its last event first. */
int radsort_last_stats(radsort_stats* out);

/* Text for a return code (and, after RADSORT_E_DEVICE, the HIP error). */
const char* radsort_strerror(int code);

/* ---------------------------------------------------------------------------
 * Step interface: the Radsort state (A, T, pi, P, f of Sec. 2.1) kept between
 * calls.  It runs the phases one at a time, exposes the permuted representation
 * between rounds (Sec. 4.1: the data can be read in logical order without
 * finalizing), and lets tests compare every round with the sequential algorithm.
 * ------------------------------------------------------------------------- */
typedef struct radsort_state radsort_state;

/* Creates a state over caller-owned keys/payload (device, n elements each; they
 * must outlive the state).  Allocates the workspace unless opts->workspace is
 * given.  Nothing is enqueued. */
int radsort_state_create(radsort_state** out, void* keys, void* payload, uint64_t n,
                         int key_bytes, int payload_bytes, int digit_bits,
                         const radsort_opts* opts);
/* Enqueues setup (Alg. 4): pi, the tail block in T, P and f. */
int radsort_state_setup(radsort_state* st, void* stream);
/* Enqueues the next round: the digit counts of the round's input (read through
 * the permuted representation), the closed forms of Alg. 5 and 6 from them (C,
 * the bucket starts S, the next P and f), the sort phase (Alg. 5) and the fixup
 * phase (Alg. 6).  Rounds run t = n_t-1 first; at most n_t rounds per setup or
 * restart. */
int radsort_state_round(radsort_state* st, void* stream);
/* Enqueues finalize (Alg. 7): the dataset ends in logical order in keys[0 .. c)
 * and payload[0 .. c), c = radsort_state_count (n unless truncated; the rest of
 * the arrays is then unspecified).  The state is used up: rounds, finalize,
 * truncate, restart, the block table and the gather return RADSORT_E_INVALID
 * until the next setup. */
int radsort_state_finalize(radsort_state* st, void* stream);
/* Finalize by the one-workgroup sequential form of Alg. 7 (slow; a test aid).
 * RADSORT_E_UNSUPPORTED after a truncate. */
int radsort_state_finalize_sequential(radsort_state* st, void* stream);
/* Waits for the stream and copies the state to host memory: pi (n_pi uint32),
 * P (sigma logical indices and sigma lengths, uint32) and f.  Any of the output
 * pointers may be NULL.  Returns RADSORT_E_TIMEOUT if a device-side check failed. */
int radsort_state_read(radsort_state* st, uint32_t* pi, uint32_t* P_idx, uint32_t* P_len,
                       uint32_t* f, void* stream);
/* Enqueues a gather of the used elements of logical blocks sigma .. f-1 in
 * logical order (data invariant, clause 5) into device arrays keys_out /
 * payload_out of radsort_state_count elements each. */
int radsort_state_logical(radsort_state* st, void* keys_out, void* payload_out,
                          void* stream);

/* ---- using the sorted data without finalize (Sec. 4.1) ----------------------
 * Between rounds, and after the last one, the dataset can be read and changed
 * in place through the permuted representation, cut short (Alg. 8), and sorted
 * again from the same state, with no finalize and no new setup.  All of these
 * are enqueued on `stream` and allocate nothing. */

/* Enqueues the block table of the permuted representation into device arrays of
 * n_pi - sigma uint32 words (either may be NULL, not both): for logical block
 * L = sigma .. n_pi - 1, phys[L - sigma] is its physical block pi[L] and
 * len[L - sigma] its used length; unallocated blocks (L >= f) give phys =
 * 0xFFFFFFFF and len = 0.  The k-th element of the dataset is element o of the
 * block that holds it (logical order, Sec. 2.2 clause 5); physical block p starts
 * at element p * b of the scratch planes (radsort_state_planes) if p < 2 sigma,
 * else at element (p - 2 sigma) * b of the caller's keys/payload (blockat, Eq. 1).
 * Keys and payloads may be rewritten there in place; the next round, or a
 * restart, reads what is there. */
int radsort_state_blocks(radsort_state* st, uint32_t* phys, uint32_t* len, void* stream);
/* The device addresses of the scratch planes T (keys, and payload or NULL) and
 * the block size b in elements.  The planes belong to the state. */
int radsort_state_planes(const radsort_state* st, void** t_keys, void** t_payload,
                         uint32_t* block_elems);
/* Elements in the dataset: n after create and setup, fewer after a truncate
 * (also after the finalize that follows it). */
int radsort_state_count(const radsort_state* st, uint64_t* count);
/* truncate (Alg. 8): keeps the first `count` elements of the dataset in its
 * current logical order (count = 0 empties it).  Allowed after setup and between
 * rounds; the rounds still to run then sort the shorter dataset, and so does a
 * later restart.  Enqueues one small kernel that finds the block and offset of
 * element count-1 and changes f and P as Alg. 8 does.  Returns RADSORT_E_INVALID
 * (state unchanged) if count exceeds radsort_state_count or the state is not set
 * up. */
int radsort_state_truncate(radsort_state* st, uint64_t count, void* stream);
/* Starts a new sort of the current contents from the current state (the state
 * becomes the input of round 0; another n_t rounds may run): for data changed
 * in place or truncated since the last sort, with no finalize and no setup.
 * Enqueues a copy of P and f (2 sigma + 1 words). */
int radsort_state_restart(radsort_state* st, void* stream);
/* n_pi, sigma and n_t of the state. */
int radsort_state_dims(const radsort_state* st, uint32_t* npi, uint32_t* sigma,
                       uint32_t* nt);
/* Frees the state and the workspace it allocated (call after the stream is done). */
int radsort_state_destroy(radsort_state* st);

/* A plain device-to-device copy of `bytes` (16-byte aligned device pointers that do
 * not overlap), enqueued on `stream`: the streaming-copy rate is the practical HBM
 * ceiling against which the sort's passes are measured (the paper's parallel sort
 * is bounded by the memory channels, Sec. 4.3).  Returns RADSORT_E_INVALID for a
 * null or unaligned pointer with bytes > 0. */
int radsort_copy(void* dst, const void* src, uint64_t bytes, void* stream);

/* MSD-first split (Sec. 4.3, last paragraph): one Radsort round on the most
 * significant digit, then finalize, which leaves the array grouped by that digit;
 * then every group is sorted by the remaining digits as one batch of independent
 * arrays (radsort_sort_segments).  The result equals radsort_sort_pairs'.
 * Arguments as radsort_sort_pairs; opts->workspace must be NULL (the library
 * allocates each phase's workspace and frees it: the peak is the larger of the
 * round's workspace and the batch's, reported by radsort_last_stats), and the
 * call waits for the stream once, between the two phases, to read the group
 * sizes.  Errors as radsort_sort_pairs. */
int radsort_msd_sort_pairs(void* keys, void* payload, uint64_t n, int key_bytes,
                           int payload_bytes, int digit_bits, const radsort_opts* opts,
                           void* stream);

/* ---- for callers that cannot allocate ------------------------------------------
 * For code under HIP graph capture, tight serving loops and harnesses that forbid
 * device allocation: radsort_sort_pairs with its workspace taken from a static
 * device array of the library, RADSORT_NOALLOC_SCRATCH_BYTES per GPU, held by every
 * GPU the library runs on until the process ends.  The call allocates nothing, on
 * the device or the host (it makes no hipMalloc, hipFree, event or state
 * allocation).  Arguments as radsort_sort_pairs, with block_elems (b, 0 selects
 * 1024) and flags (RADSORT_F_CHECK, RADSORT_F_SEQ_DRAWS; RADSORT_F_TIMING, which
 * creates events, is rejected with RADSORT_E_INVALID) given directly.  A sort whose
 * workspace (radsort_workspace_bytes) exceeds the static array returns
 * RADSORT_E_NOMEM before anything is enqueued; for 8-bit digits and b = 2048 the
 * array holds the workspace of up to about 2^28 uint32 key + uint32 payload pairs.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other threads) race and give undefined results; calls ordered on
 * one stream are safe, each clearing what it needs. */
#define RADSORT_NOALLOC_SCRATCH_BYTES (32ull << 20)
int radsort_sort_pairs_noalloc(void* keys, void* payload, uint64_t n, int key_bytes,
                               int payload_bytes, int digit_bits, uint32_t block_elems,
                               uint32_t flags, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RADSORT_H */
