/*
 * vmt_oracle.h -- plain scalar CPU reference for the V-family generators.
 *
 * TEST INFRASTRUCTURE. This library is the oracle that the HIP path is
 * checked against. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product library never does, and the
 * two share no code, header, table or constant generator.
 *
 * Source: F. Cannizzo, "VMT19937: A SIMD-Friendly Pseudo Random Number
 * Generator based on Mersenne Twister 19937" (arXiv 2309.16682).
 *   - Sec. 2.1, eq. (step), (matmult), (tempering): the MT recurrence template.
 *   - Sec. 2.2 eq. (params) and Sec. 2.3 eq. (params64): MT19937-32/-64 constants.
 *   - Sec. 2.4 eq. (sfmt_step), (sfmt_params): the SFMT19937 recurrence.
 *   - Sec. 2.5 eq. (staterec), (stepmod): the circular-buffer state.
 *   - Sec. 3 eq. (subseq), (combseq) and Table (jvalues): the interleaved
 *     V-stream, lane t = the base stream advanced by t*J steps.
 *   - Sec. 3.1: jump-ahead (state after J steps = a linear map of the state).
 *
 * Everything here is deliberately the slow, obvious form: one word per step on
 * a circular buffer, bit-serial polynomial arithmetic over GF(2), Horner's rule
 * for the jump, and lanes advanced one after the other.
 *
 * Conventions
 *   variant 0 = MT19937-32, 1 = MT19937-64, 2 = SFMT19937, 3..7 = SFMT607,
 *   SFMT1279, SFMT2281, SFMT4253, SFMT11213 (the same recurrence with the
 *   generator authors' parameter sets for those Mersenne exponents).
 *   A "canonical" state lists the n words oldest first: x_k, ..., x_{k+n-1}.
 *   SFMT words are 128-bit, stored as four uint32 sub-words, sub-word 0 the
 *   least significant (value = sum_j w^(j) 2^(32 j)).
 *   A GF(2) polynomial is an array of OR_PW uint64 words, bit i of the
 *   array = coefficient of t^i.
 *
 * Parity notes (readings where the paper is silent) are listed with each
 * function in vmt_oracle.c.
 */
#ifndef VMT_ORACLE_H
#define VMT_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_PW 640 /* words per polynomial buffer (40960 coefficients) */

/* ---- base generators (scalar, circular buffer) --------------------------- */

/* Number of state words n, the byte size of one word, and the Mersenne
 * exponent (the period is a multiple of 2^MEXP - 1) of a variant. */
int or_state_words(int variant);
int or_word_bytes(int variant);
int or_mexp(int variant);

/* Seeding. The paper does not give a seeding procedure; these follow the
 * published initialisations of the base generators (see vmt_oracle.c). */
void or_mt32_init_genrand(uint32_t x[624], uint32_t seed);
void or_mt32_init_by_array(uint32_t x[624], const uint32_t* key, int key_len);
void or_mt64_init_genrand(uint64_t x[312], uint64_t seed);
/* SFMT of any variant >= 2: x holds 4N uint32. Returns 1 if period
 * certification flipped a bit, 0 if not. or_sfmt_init_genrand is SFMT19937. */
int or_sfmt_init(int variant, uint32_t* x, uint32_t seed);
int or_sfmt_init_genrand(uint32_t x[624], uint32_t seed);
/* The period-certification vector of an SFMT variant. */
void or_sfmt_parity(int variant, uint32_t parity[4]);

/* Tempering g() of eq. (tempering). */
uint32_t or_mt32_temper(uint32_t y);
uint64_t or_mt64_temper(uint64_t y);

/* Advance a circular-buffer state by `count` recurrence steps. buf holds the
 * n words; *k is the slot of the oldest word. If out is not NULL it receives
 * the new words: raw (temper=0) or tempered (temper=1; ignored for SFMT,
 * which has no tempering). SFMT writes 4 uint32 per step. */
void or_step(int variant, void* buf, int* k, void* out, size_t count, int temper);

/* Rotate a circular buffer into canonical order. */
void or_canon(int variant, const void* buf, int k, void* canon);

/* ---- GF(2)[t] arithmetic --------------------------------------------------- */

int or_poly_deg(const uint64_t* a);                                     /* -1 for 0 */
void or_poly_mod(uint64_t* a, const uint64_t* mu);                      /* a := a mod mu */
void or_poly_mulmod(uint64_t* r, const uint64_t* a, const uint64_t* b, const uint64_t* mu);
void or_poly_sqrmod(uint64_t* r, const uint64_t* a, const uint64_t* mu);
/* r := t^(2^k) mod mu by k squarings starting from start (or from t if start is NULL). */
void or_poly_sqr_chain(uint64_t* r, const uint64_t* start, uint64_t k, const uint64_t* mu);
/* r := t^e mod mu; e is a little-endian multiword integer. */
void or_poly_powmod_t(uint64_t* r, const uint64_t* e, int e_words, const uint64_t* mu);
void or_poly_gcd(uint64_t* r, const uint64_t* a, const uint64_t* b);

/* Minimal polynomial (shortest linear recurrence) of an arbitrary bit
 * sequence s[0..N-1] (one bit per byte, bit 0 used) by Berlekamp-Massey, in
 * characteristic orientation: sum_j poly_j s_{i+j} = 0 for every i with
 * i + L < N, L its degree = the linear complexity of the sequence. poly has
 * poly_words words; returns L, or -1 if L does not fit. */
int or_berlekamp_massey(const uint8_t* s, size_t N, uint64_t* poly, size_t poly_words);

/* Minimal polynomial of the bit sequence (bit 0 of sub-word 0 of each new raw
 * word) produced from the canonical state, by Berlekamp-Massey over
 * 2*maxdeg+64 terms. Returns its degree. */
int or_minpoly(int variant, const void* canon, uint64_t* mu);

/* Minimal polynomial of the sequence <mask, X_i> of a state's successors X_i
 * (mask: a bit mask with the canonical state's layout, as uint32). Returns its
 * degree. The lcm over a few random masks and states is the minimal
 * polynomial of the one-step map. */
int or_minpoly_masked(int variant, const void* canon, const uint32_t* mask, uint64_t* mu);

/* ---- jump ahead ------------------------------------------------------------ */

/* State := g(F) state by Horner's rule, where F is one recurrence step acting
 * on the canonical state. With g = t^d mod (minimal polynomial) this is the
 * state after d steps (Sec. 3.1). Canonical in, canonical out. */
void or_jump(int variant, void* canon, const uint64_t* g);

/* ---- the V-stream (Sec. 3) ------------------------------------------------- */

typedef struct or_vgen or_vgen;

/* M lanes: lane 0 = canon0, lane t = lane t-1 advanced by gJ (= t^J mod mu).
 * The stream interleaves the lanes' outputs round robin, eq. (combseq);
 * for SFMT the round robin is over 128-bit words and the uint32 stream lists
 * the four sub-words of each word in order. */
or_vgen* or_vgen_new(int variant, int M, const void* canon0, const uint64_t* gJ);
void or_vgen_free(or_vgen* v);
/* Next `count` stream elements: uint32 (MT32, SFMT) or uint64 (MT64). */
void or_vgen_generate(or_vgen* v, void* out, size_t count);
/* Every lane advances by g (= t^d mod mu): the stream skips d*M words. */
void or_vgen_jump(or_vgen* v, const uint64_t* g);
/* Stream position in output elements (uint32 for SFMT). */
uint64_t or_vgen_pos(const or_vgen* v);
/* Copy lane t's canonical state and the lane's pending SFMT word state. */
void or_vgen_lane_canon(const or_vgen* v, int t, void* canon);

/* ---- fixed integer-to-float maps ---------------------------------------- */
float or_u32_to_f32(uint32_t u);             /* (u >> 8) * 2^-24 */
double or_u64_to_f64(uint64_t u);            /* (u >> 11) * 2^-53 */
float or_u64_to_f32(uint64_t u);             /* (u >> 40) * 2^-24 */
double or_u32pair_to_f64(uint32_t a, uint32_t b); /* ((a>>5) 2^26 + (b>>6)) 2^-53 */
void or_map_f32(const uint32_t* u, float* f, size_t n);
void or_map_f64(const uint64_t* u, double* f, size_t n);

#ifdef __cplusplus
}
#endif
#endif
