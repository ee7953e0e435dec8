/*
 * Radsort oracle: declarations.  TEST INFRASTRUCTURE ONLY (see radsort_oracle.c).
 * This header belongs to the oracle alone; the GPU library has its own.
 */
#ifndef RADSORT_ORACLE_H
#define RADSORT_ORACLE_H

#include <stdint.h>

typedef struct { uint64_t key, val; } orc_elem;
typedef struct orc_state orc_state;

/* Counters kept by the oracle.  Indices below ORC_C_FIRST_ERROR are statistics;
 * the rest count broken assertions and must stay zero. */
enum {
    ORC_C_ROUNDS = 0,
    ORC_C_LEMMA1_EQUAL,          /* draws with i_out == i_in at the end of block i_in */
    ORC_C_FINALIZE_COPIES,       /* block copies made by finalize (push and pull) */
    ORC_C_FIRST_ERROR,
    ORC_C_LEMMA1_VIOLATION = ORC_C_FIRST_ERROR,
    ORC_C_LEMMA2_VIOLATION,
    ORC_C_POOL_OVERRUN,
    ORC_C_FINALIZE_TAIL_OVERWRITTEN, /* a tail block sat where the tail copies write */
    ORC_C_FINALIZE_COUNT_MISMATCH,
    ORC_C_FINALIZE_HOME_TAKEN,   /* a home already held a placed block */
    ORC_NCOUNTERS
};

uint64_t orc_key(uint64_t x, uint64_t t, uint64_t sigma, uint64_t nt);

orc_state *orc_create(uint64_t n, uint64_t sigma, uint64_t nt, uint64_t b);
void orc_destroy(orc_state *st);
void orc_load(orc_state *st, const uint64_t *keys, const uint64_t *vals);
void orc_store(const orc_state *st, uint64_t *keys, uint64_t *vals);
void orc_setup(orc_state *st);
void orc_sort_phase(orc_state *st, uint64_t t);
void orc_fixup_phase(orc_state *st);
void orc_round(orc_state *st, uint64_t t);
void orc_finalize(orc_state *st);
int orc_radsort(uint64_t *keys, uint64_t *vals, uint64_t n, uint64_t sigma, uint64_t nt,
                uint64_t b);

uint64_t orc_npi(const orc_state *st);
uint64_t orc_f(const orc_state *st);
uint64_t orc_i_out(const orc_state *st);
void orc_get_pi(const orc_state *st, uint64_t *out);
void orc_get_P(const orc_state *st, uint64_t *idx, uint64_t *len);
void orc_get_C(const orc_state *st, uint64_t *out);
void orc_get_counters(const orc_state *st, uint64_t *out);
uint64_t orc_get_logical(orc_state *st, uint64_t *keys, uint64_t *vals);
int orc_check_invariant(orc_state *st);
int orc_truncate(orc_state *st, uint64_t i, int64_t j);
int orc_truncate_count(orc_state *st, uint64_t count);
void orc_set_logical(orc_state *st, const uint64_t *keys, const uint64_t *vals);
uint64_t orc_n(const orc_state *st);
/* test hooks: overwrite one entry of pi or P, or f, to plant a broken state */
void orc_test_set_pi(orc_state *st, uint64_t i, uint64_t v);
void orc_test_set_P(orc_state *st, uint64_t k, uint64_t idx, uint64_t len);
void orc_test_set_f(orc_state *st, uint64_t f);

int orc_oop_lsd(uint64_t *keys, uint64_t *vals, uint64_t n, uint64_t sigma, uint64_t nt,
                uint64_t rounds);
void orc_histograms(const uint64_t *keys, uint64_t n, uint64_t sigma, uint64_t nt,
                    uint64_t *out);
uint64_t orc_extra_bytes(uint64_t n, uint64_t sigma, uint64_t b, uint64_t elem_bytes,
                         uint64_t ptr_bytes, uint64_t int_bytes);

#endif
