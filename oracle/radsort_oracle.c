/*
 * Radsort oracle: a plain, sequential CPU implementation of the LSD radix sort
 * with O(sqrt n) extra space from "Parallel O(sqrt n) Overhead LSD Radix Sort"
 * (Clausecker, Schintke).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the GPU implementation.
 *
 * What it follows (paper sections, algorithms, equations):
 *   - key(x, t): the n_t-tuple view of a key (Sec. 1).  Position t = n_t-1 is the
 *     least significant digit and is sorted first (Alg. 2).
 *   - blockat (Eq. 1), the state table and the data invariant (Sec. 2.1, 2.2).
 *   - setup (Alg. 4), sizeOfNextBlock (Alg. 3), newBucketBlock and sortPhase
 *     (Alg. 5), fixupPhase (Alg. 6), swap and finalize (Alg. 7).
 *   - truncate (Alg. 8) and use of the permuted representation without
 *     finalize (Sec. 4.1).
 *   - radixSortStep, the out-of-place round (Alg. 1).
 *   - the space formula of Sec. 3 and the worked overhead numbers of Sec. 4.
 *
 * Readings taken where the printed text is ambiguous or garbled (each is also
 * listed in the design notes of the repository):
 *   G1  sizeOfNextBlock (Alg. 3) compares the LOGICAL index i with P's logical
 *       index, not pi[i]: P stores logical indices (Sec. 2.1, Alg. 4, Alg. 6).
 *   G2  finalize (Alg. 7): the physical home of logical block i_in is
 *       i_in + sigma (logical sigma is the first A block, physical 2 sigma,
 *       Eq. 1), not i_in - sigma.
 *   G3  swap (Alg. 7) re-binds the (logical, physical) handle pairs so that each
 *       pair keeps naming one block (Eq. 4); the loop counter i_in of finalize
 *       is never changed by it, and the free slot becomes the block pulled from.
 *   G4  setup: data lives at logical sigma .. sigma+floor(n/b)-1 and the tail
 *       (n mod b elements, possibly zero) at logical f-1 = physical sigma.
 *   G5  eager allocation: a bucket's next block is drawn as soon as its current
 *       block becomes full (Alg. 5), so a bucket ends with a block that may be
 *       empty; its partial length is in [0, b).
 *   G7  integer keys: unsigned, ascending; digits by shift/mask for power-of-two
 *       alphabets, by division for other alphabets; sigma is the same in every
 *       round even when the top digit has fewer significant bits.
 *   G13 truncate (Alg. 8) leaves the entries of P after the one it rewrites;
 *       they name blocks at or beyond the new f and are inactive.  The final block
 *       may then be full (length b) and is still tracked in P.
 *   G14 finalize after truncate: the element count is the truncated one, and a
 *       block of the tail that sits in the A block right after the homes is first
 *       moved to a free block of T (the tail copies write into that A block).
 *
 * Lemma 1 is asserted in its tight form: when a bucket takes a new block during
 * the scan, the pool entry it takes lies before the input block being read, or is
 * that block when the element just written was its last one (the block has then
 * been read completely).
 */
#include "radsort_oracle.h"

#include <stdlib.h>
#include <string.h>

struct orc_state {
    /* state table (Sec. 2.1) */
    uint64_t n, sigma, nt, b, npi;
    orc_elem *A;        /* the array being sorted, n elements */
    orc_elem *T;        /* 2 sigma b scratch elements */
    uint64_t f;         /* fill level */
    uint64_t *pi;       /* logical -> physical block, n_pi entries */
    uint64_t *Pi, *Pl;  /* partial blocks: logical index and length, sigma entries */
    /* round temporaries (Sec. 2.3), kept in this oracle's own form: the blocks a
     * round takes are numbered by their place in the pool pi[0], pi[1], ...; each
     * bucket has a cursor (the pool entry of the block it is filling and how many
     * elements that block holds); owner[h] is the bucket that took pool entry h;
     * blocks_of[c] counts the blocks bucket c took; taken counts the pool entries
     * handed out so far. */
    uint64_t *cur_entry, *cur_fill, *blocks_of, *start;
    uint32_t *owner;
    uint64_t *pi2;
    uint64_t taken;
    /* finalize temporaries (Sec. 2.4) */
    uint64_t *pinv;
    /* instrumentation */
    uint64_t counters[ORC_NCOUNTERS];
};

/* ---- keys (Sec. 1; digit extraction by shift and mask, Sec. 4) ---------------- */

static int is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

static uint64_t log2u(uint64_t x)
{
    uint64_t r = 0;
    while ((1ull << r) < x) r++;
    return r;
}

/* key(x, t): digit t of the n_t-digit base-sigma representation of x, where
 * t = 0 is the most significant digit. */
uint64_t orc_key(uint64_t x, uint64_t t, uint64_t sigma, uint64_t nt)
{
    uint64_t below = nt - 1 - t; /* number of less significant digits */
    if (is_pow2(sigma)) {
        uint64_t shift = below * log2u(sigma);
        if (shift >= 64) return 0;
        return (x >> shift) & (sigma - 1);
    }
    for (uint64_t k = 0; k < below; k++) x /= sigma;
    return x % sigma;
}

/* ---- blocks (Eq. 1) ------------------------------------------------------------- */

static orc_elem *blockat(orc_state *st, uint64_t i)
{
    if (i < 2 * st->sigma) return st->T + i * st->b;
    return st->A + (i - 2 * st->sigma) * st->b;
}

/* ---- life cycle ----------------------------------------------------------------- */

orc_state *orc_create(uint64_t n, uint64_t sigma, uint64_t nt, uint64_t b)
{
    if (sigma < 2 || nt < 1 || b < 1) return NULL;
    orc_state *st = calloc(1, sizeof *st);
    if (!st) return NULL;
    st->n = n;
    st->sigma = sigma;
    st->nt = nt;
    st->b = b;
    st->npi = n / b + 2 * sigma; /* state table, Sec. 2.1 */
    st->A = calloc(n ? n : 1, sizeof(orc_elem));
    st->T = calloc(2 * sigma * b, sizeof(orc_elem));
    st->pi = calloc(st->npi, sizeof(uint64_t));
    st->pi2 = calloc(st->npi, sizeof(uint64_t));
    st->pinv = calloc(st->npi, sizeof(uint64_t));
    st->owner = calloc(st->npi, sizeof(uint32_t));
    st->Pi = calloc(sigma, sizeof(uint64_t));
    st->Pl = calloc(sigma, sizeof(uint64_t));
    st->cur_entry = calloc(sigma, sizeof(uint64_t));
    st->cur_fill = calloc(sigma, sizeof(uint64_t));
    st->blocks_of = calloc(sigma, sizeof(uint64_t));
    st->start = calloc(sigma, sizeof(uint64_t));
    if (!st->A || !st->T || !st->pi || !st->pi2 || !st->pinv || !st->owner || !st->Pi ||
        !st->Pl || !st->cur_entry || !st->cur_fill || !st->blocks_of || !st->start) {
        orc_destroy(st);
        return NULL;
    }
    return st;
}

void orc_destroy(orc_state *st)
{
    if (!st) return;
    free(st->A); free(st->T); free(st->pi); free(st->pi2); free(st->pinv);
    free(st->owner); free(st->Pi); free(st->Pl); free(st->cur_entry); free(st->cur_fill);
    free(st->blocks_of); free(st->start);
    free(st);
}

void orc_load(orc_state *st, const uint64_t *keys, const uint64_t *vals)
{
    for (uint64_t i = 0; i < st->n; i++) {
        st->A[i].key = keys[i];
        st->A[i].val = vals ? vals[i] : 0;
    }
}

void orc_store(const orc_state *st, uint64_t *keys, uint64_t *vals)
{
    for (uint64_t i = 0; i < st->n; i++) {
        keys[i] = st->A[i].key;
        if (vals) vals[i] = st->A[i].val;
    }
}

/* ---- setup (Alg. 4) --------------------------------------------------------------- */

void orc_setup(orc_state *st)
{
    uint64_t sigma = st->sigma, b = st->b, n = st->n;
    st->f = sigma + n / b + 1;
    for (uint64_t i = 0; i < sigma; i++) st->pi[i] = i;                 /* head start */
    for (uint64_t i = sigma; i + 1 < st->f; i++) st->pi[i] = i + sigma;  /* blocks of A */
    for (uint64_t i = st->f - 1; i < st->npi; i++)                       /* the rest, in T */
        st->pi[i] = sigma + (i - (st->f - 1));
    memset(st->T, 0, 2 * sigma * b * sizeof(orc_elem));                  /* dummy fill */
    memcpy(blockat(st, sigma), st->A + b * (n / b), (n % b) * sizeof(orc_elem));
    st->Pi[0] = st->f - 1;                                               /* the tail */
    st->Pl[0] = n % b;
    for (uint64_t i = 1; i < sigma; i++) {                               /* dummies */
        st->Pi[i] = st->npi;
        st->Pl[i] = 0;
    }
}

/* ---- sizeOfNextBlock (Alg. 3, reading G1) ---------------------------------------- */

static uint64_t size_of_next_block(const orc_state *st, uint64_t i, uint64_t *iP)
{
    if (*iP < st->sigma && st->Pi[*iP] == i) {
        uint64_t l = st->Pl[*iP];
        (*iP)++;
        return l;
    }
    return st->b;
}

/* ---- sortPhase with newBucketBlock (Alg. 5) --------------------------------------
 *
 * The pool is pi read in logical order: its first sigma entries are the head
 * start, then come the input blocks sigma .. f-1, then the unallocated ones.  A
 * bucket holds one open block at a time; when that block has received b elements
 * the bucket takes the next pool entry (eager allocation, reading G5).  Lemma 1
 * says the entry taken then is an input block the scan has already passed. */

/* Hands bucket c the next pool entry as its open, empty block.  Returns 0 when
 * the pool is exhausted (never for a correct state: Lemma 1); the scan then stops
 * and the round's state is not usable. */
static int give_block(orc_state *st, uint64_t c)
{
    if (st->taken >= st->npi) { st->counters[ORC_C_POOL_OVERRUN]++; return 0; }
    st->cur_entry[c] = st->taken;
    st->cur_fill[c] = 0;
    st->owner[st->taken] = (uint32_t)c;
    st->blocks_of[c]++;
    st->taken++;
    return 1;
}

void orc_sort_phase(orc_state *st, uint64_t t)
{
    const uint64_t sigma = st->sigma, b = st->b;
    st->taken = 0;
    for (uint64_t c = 0; c < sigma; c++) st->blocks_of[c] = 0;
    for (uint64_t c = 0; c < sigma; c++)    /* every bucket starts in its head-start block */
        if (!give_block(st, c)) return;
    uint64_t iP = 0;
    for (uint64_t L = sigma; L < st->f; L++) {            /* input blocks in logical order */
        const uint64_t len = size_of_next_block(st, L, &iP);
        const orc_elem *in = blockat(st, st->pi[L]);
        for (uint64_t j = 0; j < len; j++) {
            const uint64_t c = orc_key(in[j].key, t, st->sigma, st->nt);
            orc_elem *out = blockat(st, st->pi[st->cur_entry[c]]);
            out[st->cur_fill[c]] = in[j];
            st->cur_fill[c]++;
            if (st->cur_fill[c] < b) continue;
            /* the block is full: the bucket needs the next pool entry.  Lemma 1, tight
             * form: that entry is a block the scan has left, or the current input
             * block L when this element was its last one. */
            if (st->taken == L && j + 1 == len) st->counters[ORC_C_LEMMA1_EQUAL]++;
            else if (st->taken >= L) st->counters[ORC_C_LEMMA1_VIOLATION]++;
            if (!give_block(st, c)) return;
        }
    }
}

/* ---- fixupPhase (Alg. 6) -------------------------------------------------------------
 *
 * The new logical order lists the buckets one after the other behind a fresh head
 * start: bucket c's blocks, in the order it took them, go to logical indices
 * start[c] .. start[c] + blocks_of[c] - 1 with start[c] = sigma + the blocks of
 * the buckets before c.  Each bucket's last block is the one it is still
 * filling, which becomes its partial block in P.  The next sigma pool entries
 * after the taken ones become the head start; entries past them stay where they
 * are.  Lemma 2 says at least sigma entries are left for that head start. */
void orc_fixup_phase(orc_state *st)
{
    const uint64_t sigma = st->sigma, npi = st->npi, taken = st->taken;
    if (npi < taken + sigma) {                           /* Lemma 2 */
        st->counters[ORC_C_LEMMA2_VIOLATION]++;
        return;
    }
    uint64_t next_free = sigma;
    for (uint64_t c = 0; c < sigma; c++) {
        st->start[c] = next_free;
        next_free += st->blocks_of[c];
    }
    for (uint64_t c = 0; c < sigma; c++) {               /* partial block of each bucket */
        st->Pi[c] = st->start[c] + st->blocks_of[c] - 1;
        st->Pl[c] = st->cur_fill[c];
    }
    for (uint64_t h = 0; h < taken; h++) {               /* blocks in bucket order */
        const uint64_t c = st->owner[h];
        st->pi2[st->start[c]++] = st->pi[h];
    }
    for (uint64_t k = 0; k < sigma; k++) st->pi2[k] = st->pi[taken + k];   /* head start */
    for (uint64_t L = taken + sigma; L < npi; L++) st->pi2[L] = st->pi[L]; /* unallocated */
    st->f = taken + sigma;
    uint64_t *tmp = st->pi;
    st->pi = st->pi2;
    st->pi2 = tmp;
}

void orc_round(orc_state *st, uint64_t t)
{
    orc_sort_phase(st, t);
    orc_fixup_phase(st);
    st->counters[ORC_C_ROUNDS]++;
}

/* ---- finalize (Alg. 7, readings G2, G3 and G14) ----------------------------------
 *
 * The sorted sequence is the used part of logical blocks sigma .. f-1, in logical
 * order.  It is packed into A from the front; `placed` counts the elements already
 * there.  The walk gives each of the first floor(n/b) logical blocks L, for keeps,
 * the physical block L + sigma (block L - sigma of A, reading G2) and appends L's
 * elements at A[placed ..].  That range ends inside L's new block, so the only live
 * data it can hit is what that block held: if the block holds a block of the
 * sequence the walk has not reached, that block is first copied to a spare block
 * (one that holds no live data) and re-bound there.  After the append, the block L
 * came from holds nothing live and becomes the spare (reading G3).  The blocks past
 * the first floor(n/b) then all sit in T, or, after a truncate, also right behind
 * the homes (reading G14), and are appended in order.  pi and its inverse follow
 * every move, so the state stays the permuted representation of the data. */

typedef struct {
    uint64_t logical, phys;  /* a physical block without live data, and its binding */
} orc_spare;

/* Binds logical block i to physical block j in pi and in its inverse. */
static void bind(orc_state *st, uint64_t i, uint64_t j)
{
    st->pi[i] = j;
    st->pinv[j] = i;
}

/* Physical block `home` holds a block of the sequence that is still to come: copy it
 * to the spare and exchange the two bindings.  Returns the logical index now bound
 * to `home`, which holds nothing live. */
static uint64_t evacuate(orc_state *st, uint64_t home, const orc_spare *spare)
{
    const uint64_t later = st->pinv[home];
    memcpy(blockat(st, spare->phys), blockat(st, home), st->b * sizeof(orc_elem));
    st->counters[ORC_C_FINALIZE_COPIES]++;
    bind(st, later, spare->phys);
    bind(st, spare->logical, home);
    return spare->logical;
}

/* Appends the used elements of logical block L, held by physical block `from`, to the
 * packed prefix of A.  Returns 0 when the lengths add up to more than n (a broken
 * state: nothing more is moved). */
static int append(orc_state *st, uint64_t L, uint64_t from, uint64_t *placed, uint64_t *iP)
{
    const uint64_t len = size_of_next_block(st, L, iP);
    if (*placed + len > st->n) {
        st->counters[ORC_C_FINALIZE_COUNT_MISMATCH]++;
        return 0;
    }
    memmove(st->A + *placed, blockat(st, from), len * sizeof(orc_elem));
    st->counters[ORC_C_FINALIZE_COPIES]++;
    *placed += len;
    return 1;
}

/* Reading G14: after a truncate A has more blocks than the floor(n/b) homes, and the
 * physical block right behind the homes may hold a block of the remaining sequence,
 * which the appends of the earlier remaining blocks would overwrite before it is
 * read.  It moves to a block of T without live data (T holds at most sigma blocks of
 * the sequence at this point, so one is free). */
static void clear_behind_homes(orc_state *st, uint64_t homes)
{
    const uint64_t sigma = st->sigma, behind = 2 * sigma + homes;
    if (behind >= st->npi) return;
    const uint64_t occupant = st->pinv[behind];
    if (occupant < sigma + homes || occupant >= st->f) return;
    uint64_t t = 0;
    while (t < 2 * sigma && st->pinv[t] >= sigma && st->pinv[t] < st->f) t++;
    if (t == 2 * sigma) {
        st->counters[ORC_C_FINALIZE_TAIL_OVERWRITTEN]++;
        return;
    }
    const uint64_t idle = st->pinv[t];
    memcpy(blockat(st, t), blockat(st, behind), st->b * sizeof(orc_elem));
    st->counters[ORC_C_FINALIZE_COPIES]++;
    bind(st, occupant, t);
    bind(st, idle, behind);
}

void orc_finalize(orc_state *st)
{
    const uint64_t sigma = st->sigma, homes = st->n / st->b;
    uint64_t placed = 0, iP = 0;
    orc_spare spare = {0, st->pi[0]};  /* logical block 0 is unallocated (Sec. 2.2) */
    for (uint64_t i = 0; i < st->npi; i++) st->pinv[st->pi[i]] = i;
    for (uint64_t L = sigma; L < sigma + homes; L++) {
        const uint64_t home = L + sigma, from = st->pi[L];
        uint64_t bound_there = st->pinv[home];
        /* a block the walk has already placed can never sit at a later home */
        if (bound_there >= sigma && bound_there < L) st->counters[ORC_C_FINALIZE_HOME_TAKEN]++;
        if (bound_there > L && bound_there < st->f) bound_there = evacuate(st, home, &spare);
        if (!append(st, L, from, &placed, &iP)) return;
        /* L keeps `home`; the index bound there takes L's old block, now without live data */
        bind(st, L, home);
        bind(st, bound_there, from);
        if (from != home) {
            spare.logical = bound_there;
            spare.phys = from;
        }
    }
    clear_behind_homes(st, homes);
    for (uint64_t L = sigma + homes; L < st->f; L++) {
        const uint64_t from = st->pi[L];
        /* the appends write A[placed .. n); a block of A they read must lie past that */
        if (from >= 2 * sigma && from - 2 * sigma <= homes)
            st->counters[ORC_C_FINALIZE_TAIL_OVERWRITTEN]++;
        if (!append(st, L, from, &placed, &iP)) return;
    }
    if (placed != st->n) st->counters[ORC_C_FINALIZE_COUNT_MISMATCH]++;
}

/* ---- truncate (Alg. 8) and writing through the permuted representation (Sec. 4.1) -- */

/* truncate(i, j): element j of logical block i becomes the last datum.  f becomes
 * i + 1, and the first entry of P whose logical index is at or after i becomes
 * (i, j + 1); the entries after it name blocks at or beyond the new f, which
 * sizeOfNextBlock never reaches, so they are left as they are (G13).  j = -1 leaves
 * block i empty; truncate(sigma, -1) empties the dataset.  The oracle also keeps
 * the element count n, which finalize and the invariant check use.  Returns 0, or
 * -1 (state unchanged) when (i, j) does not name an element of the dataset (or
 * the place before the first element of block i). */
int orc_truncate(orc_state *st, uint64_t i, int64_t j)
{
    if (i < st->sigma || i >= st->f || j < -1) return -1;
    uint64_t k = 0, iP = 0;
    for (uint64_t L = st->sigma; L < i; L++) k += size_of_next_block(st, L, &iP);
    uint64_t len_i = size_of_next_block(st, i, &iP);
    if (j >= 0 && (uint64_t)j >= len_i) return -1;
    st->f = i + 1;                                  /* block i is the final block */
    for (uint64_t e = 0; e < st->sigma; e++) {      /* skip partials before block i */
        if (i <= st->Pi[e]) {
            st->Pi[e] = i;
            st->Pl[e] = (uint64_t)(j + 1);          /* block i ends at element j */
            break;
        }
    }
    st->n = k + (uint64_t)(j + 1);
    return 0;
}

/* Keeps the first `count` elements of the logical sequence: truncate at the block
 * and offset of element count - 1, found by walking the blocks as sizeOfNextBlock
 * does (Alg. 3); count = 0 empties the dataset.  Returns -1 if count > n. */
int orc_truncate_count(orc_state *st, uint64_t count)
{
    if (count == 0) return orc_truncate(st, st->sigma, -1);
    uint64_t k = 0, iP = 0;
    for (uint64_t L = st->sigma; L < st->f; L++) {
        uint64_t l = size_of_next_block(st, L, &iP);
        if (count - 1 < k + l) return orc_truncate(st, L, (int64_t)(count - 1 - k));
        k += l;
    }
    return -1;
}

/* Overwrites the used elements of the allocated blocks, in logical order, with
 * keys[0 .. n) and vals[0 .. n) (vals may be NULL: payloads are kept): the
 * dataset modified in place through the permuted representation (Sec. 4.1). */
void orc_set_logical(orc_state *st, const uint64_t *keys, const uint64_t *vals)
{
    uint64_t k = 0, iP = 0;
    for (uint64_t i = st->sigma; i < st->f; i++) {
        orc_elem *p = blockat(st, st->pi[i]);
        uint64_t l = size_of_next_block(st, i, &iP);
        for (uint64_t j = 0; j < l && k < st->n; j++, k++) {
            p[j].key = keys[k];
            if (vals) p[j].val = vals[k];
        }
    }
}

uint64_t orc_n(const orc_state *st) { return st->n; }

/* ---- test hooks: plant a broken state for the invariant checker's pins ------------ */

void orc_test_set_pi(orc_state *st, uint64_t i, uint64_t v)
{
    if (i < st->npi) st->pi[i] = v;
}

void orc_test_set_P(orc_state *st, uint64_t k, uint64_t idx, uint64_t len)
{
    if (k < st->sigma) {
        st->Pi[k] = idx;
        st->Pl[k] = len;
    }
}

void orc_test_set_f(orc_state *st, uint64_t f) { st->f = f; }

/* ---- the driver (Alg. 2) ----------------------------------------------------------- */

int orc_radsort(uint64_t *keys, uint64_t *vals, uint64_t n, uint64_t sigma, uint64_t nt,
                uint64_t b)
{
    orc_state *st = orc_create(n, sigma, nt, b);
    if (!st) return -1;
    orc_load(st, keys, vals);
    orc_setup(st);
    for (uint64_t t = nt; t-- > 0;) orc_round(st, t);
    int bad = 0;
    for (int c = ORC_C_FIRST_ERROR; c < ORC_NCOUNTERS; c++) bad |= st->counters[c] != 0;
    if (!bad) {  /* a state whose rounds broke a lemma is not finalized */
        orc_finalize(st);
        for (int c = ORC_C_FIRST_ERROR; c < ORC_NCOUNTERS; c++) bad |= st->counters[c] != 0;
    }
    orc_store(st, keys, vals);
    orc_destroy(st);
    return bad ? -2 : 0;
}

/* ---- inspection --------------------------------------------------------------------- */

uint64_t orc_npi(const orc_state *st) { return st->npi; }
uint64_t orc_f(const orc_state *st) { return st->f; }
uint64_t orc_i_out(const orc_state *st) { return st->taken; }

void orc_get_pi(const orc_state *st, uint64_t *out)
{
    memcpy(out, st->pi, st->npi * sizeof(uint64_t));
}

void orc_get_P(const orc_state *st, uint64_t *idx, uint64_t *len)
{
    memcpy(idx, st->Pi, st->sigma * sizeof(uint64_t));
    memcpy(len, st->Pl, st->sigma * sizeof(uint64_t));
}

void orc_get_C(const orc_state *st, uint64_t *out)
{
    memcpy(out, st->blocks_of, st->sigma * sizeof(uint64_t));
}

void orc_get_counters(const orc_state *st, uint64_t *out)
{
    memcpy(out, st->counters, sizeof st->counters);
}

/* The used elements of the allocated blocks sigma .. f-1 in logical order
 * (data invariant, clause 5), found by walking P as sizeOfNextBlock does. */
uint64_t orc_get_logical(orc_state *st, uint64_t *keys, uint64_t *vals)
{
    uint64_t k = 0, iP = 0;
    for (uint64_t i = st->sigma; i < st->f; i++) {
        orc_elem *p = blockat(st, st->pi[i]);
        uint64_t l = size_of_next_block(st, i, &iP);
        for (uint64_t j = 0; j < l; j++, k++) {
            if (k < st->n) {
                keys[k] = p[j].key;
                if (vals) vals[k] = p[j].val;
            }
        }
    }
    return k;
}

/* The data invariant of Sec. 2.2, clauses 1-4 (clause 5 is checked by the tests
 * from the logical sequence).  Returns 0 when it holds, else the clause number. */
int orc_check_invariant(orc_state *st)
{
    uint64_t npi = st->npi, sigma = st->sigma;
    unsigned char *seen = calloc(npi, 1);
    if (!seen) return -1;
    int bad = 0;
    for (uint64_t i = 0; i < npi && !bad; i++) {
        if (st->pi[i] >= npi || seen[st->pi[i]]) bad = 1;
        else seen[st->pi[i]] = 1;
    }
    free(seen);
    if (bad) return 1;
    /* clause 2: real entries of P ascending and inside the allocated range */
    uint64_t prev = 0;
    int have_prev = 0;
    for (uint64_t i = 0; i < sigma; i++) {
        if (st->Pi[i] == npi) continue; /* dummy entry of setup */
        if (st->Pi[i] < sigma || (have_prev && st->Pi[i] <= prev)) return 2;
        prev = st->Pi[i];
        have_prev = 1;
        if (st->Pi[i] >= st->f) continue; /* left behind by truncate (G13) */
        /* a partial block holds fewer than b elements; after truncate the final
         * block may be full (G13) */
        if (st->Pl[i] > st->b || (st->Pl[i] == st->b && st->Pi[i] != st->f - 1)) return 2;
    }
    /* clause 3: f-1 is a partial block */
    int found = 0;
    for (uint64_t i = 0; i < sigma; i++) found |= st->Pi[i] == st->f - 1;
    if (!found) return 3;
    /* clause 4: the allocated range fits between the head start and n_pi */
    if (st->f <= sigma || st->f > npi) return 4;
    /* the used elements add up to n */
    uint64_t k = 0, iP = 0;
    for (uint64_t i = sigma; i < st->f; i++) k += size_of_next_block(st, i, &iP);
    if (k != st->n) return 5;
    return 0;
}

/* ---- out-of-place LSD (Alg. 1) ------------------------------------------------------- */

static void radix_sort_step(orc_elem *Aout, const orc_elem *A, uint64_t n, uint64_t t,
                            uint64_t sigma, uint64_t nt, uint64_t *H)
{
    for (uint64_t c = 0; c < sigma; c++) H[c] = 0;
    for (uint64_t i = 0; i < n; i++) H[orc_key(A[i].key, t, sigma, nt)]++;
    uint64_t s = 0;                                   /* S: prefix sum over H */
    for (uint64_t c = 0; c < sigma; c++) {
        uint64_t h = H[c];
        H[c] = s;
        s += h;
    }
    for (uint64_t i = 0; i < n; i++) {
        uint64_t c = orc_key(A[i].key, t, sigma, nt);
        Aout[H[c]] = A[i];
        H[c]++;
    }
}

/* Runs `rounds` out-of-place rounds, t = n_t-1, n_t-2, ... (all n_t when rounds
 * equals n_t).  Returns 0, or -1 when memory runs out. */
int orc_oop_lsd(uint64_t *keys, uint64_t *vals, uint64_t n, uint64_t sigma, uint64_t nt,
                uint64_t rounds)
{
    orc_elem *a = malloc((n ? n : 1) * sizeof(orc_elem));
    orc_elem *a2 = malloc((n ? n : 1) * sizeof(orc_elem));
    uint64_t *H = malloc(sigma * sizeof(uint64_t));
    if (!a || !a2 || !H) { free(a); free(a2); free(H); return -1; }
    for (uint64_t i = 0; i < n; i++) {
        a[i].key = keys[i];
        a[i].val = vals ? vals[i] : 0;
    }
    for (uint64_t r = 0; r < rounds && r < nt; r++) {
        radix_sort_step(a2, a, n, nt - 1 - r, sigma, nt, H);
        orc_elem *tmp = a; a = a2; a2 = tmp;
    }
    for (uint64_t i = 0; i < n; i++) {
        keys[i] = a[i].key;
        if (vals) vals[i] = a[i].val;
    }
    free(a); free(a2); free(H);
    return 0;
}

/* Histograms of every key position: out[t * sigma + c] = #{i : key(x_i, t) = c}. */
void orc_histograms(const uint64_t *keys, uint64_t n, uint64_t sigma, uint64_t nt,
                    uint64_t *out)
{
    memset(out, 0, nt * sigma * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++)
        for (uint64_t t = 0; t < nt; t++) out[t * sigma + orc_key(keys[i], t, sigma, nt)]++;
}

/* ---- extra space (Sec. 3 "Space"; worked numbers in Sec. 4) ------------------------ */

/* Bytes of storage besides A: T, then B, C, S, P, then pi, pi', U per block, with
 * pi^{-1} reusing pi'.  elem_bytes is the element size, ptr_bytes the size of a
 * pointer in B and int_bytes the size of the integers in C, S, P, pi, pi'. */
uint64_t orc_extra_bytes(uint64_t n, uint64_t sigma, uint64_t b, uint64_t elem_bytes,
                         uint64_t ptr_bytes, uint64_t int_bytes)
{
    uint64_t npi = n / b + 2 * sigma;
    uint64_t u_bytes = sigma <= 256 ? 1 : (sigma <= 65536 ? 2 : 4);
    uint64_t t_bytes = 2 * sigma * b * elem_bytes;
    uint64_t bucket_bytes = sigma * (2 * ptr_bytes + int_bytes + int_bytes + 2 * int_bytes);
    uint64_t block_bytes = npi * (2 * int_bytes + u_bytes);
    return t_bytes + bucket_bytes + block_bytes;
}
