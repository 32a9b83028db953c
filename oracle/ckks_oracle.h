/*
 * ckks_oracle.h -- plain CPU oracle of the RNS-CKKS encrypted matrix-vector
 * product with pre-rotated plaintext diagonals and the Chebyshev threshold.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant with
 * the HIP library; both sides are written independently from the paper
 * (arXiv 2604.00546) and from the published definitions they cite.
 *
 * Representation: every polynomial is kept in COEFFICIENT form, one uint64
 * word per residue, canonical in [0, q), limb-major ([limb][N]).  Polynomial
 * products go through a textbook negacyclic NTT (a library-style step); every
 * other operation is written coefficient by coefficient from its definition.
 *
 * Moduli are addressed by a global index: 0..L are the ciphertext primes
 * q_0..q_L, L+1..L+nP are the special primes p_0..p_{nP-1}.
 */
#ifndef CKKS_ORACLE_H
#define CKKS_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_ctx or_ctx;
typedef struct or_keys or_keys;
typedef struct or_db or_db;

/* A ciphertext (c0, c1): data is [2][level+1][N] coefficient-form residues. */
typedef struct or_ct {
    int level;
    double scale;
    uint64_t *c;
} or_ct;

/* A plaintext polynomial: data is [level+1][N] coefficient-form residues. */
typedef struct or_pt {
    int level;
    double scale;
    uint64_t *m;
} or_pt;

/* ---- parameters (primes chosen by the rule stated in ckks_oracle.c) ---- */
or_ctx *or_ctx_create(int logN, int q0_bits, int n_mid, int mid_bits,
                      int n_special, int special_bits, int dnum);
void or_ctx_free(or_ctx *ctx);
int or_ctx_N(const or_ctx *ctx);
int or_ctx_L(const or_ctx *ctx);
int or_ctx_nspecial(const or_ctx *ctx);
int or_ctx_alpha(const or_ctx *ctx);
uint64_t or_ctx_modulus(const or_ctx *ctx, int gidx);
const char *or_last_error(void);
/* OpenMP threads of the parallel loops (timing at a stated core count) */
void or_set_threads(int n);
int or_get_threads(void);

/* ---- randomness: Philox-4x64-10 and the three samplers ---- */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void or_gauss_cdt(uint64_t cdt[20]);
void or_sample_uniform(uint64_t seed, uint64_t poly, int gidx, uint64_t q, int N, uint64_t *out);
void or_sample_ternary(uint64_t seed, uint64_t poly, int N, int64_t *out);
void or_sample_gauss(uint64_t seed, uint64_t poly, int N, int64_t *out);
uint64_t or_galois_element(const or_ctx *ctx, int rot);

/* ---- single-modulus polynomial helpers exposed for the pins ---- */
int or_polymul(const or_ctx *ctx, int gidx, const uint64_t *a, const uint64_t *b, uint64_t *out);
void or_automorphism(const or_ctx *ctx, int gidx, uint64_t g, const uint64_t *a, uint64_t *out);
/* fast base conversion of digit t of a level-`level` polynomial x ([level+1][N])
 * to the extended basis Q_level U P: out is [level+1+nP][N]. */
int or_modup_digit(const or_ctx *ctx, int level, int t, const uint64_t *x, uint64_t *out);
/* ModDown of an extended-basis polynomial u ([level+1+nP][N]) to Q_level. */
int or_moddown(const or_ctx *ctx, int level, const uint64_t *u, uint64_t *out);

/* ---- keys ---- */
or_keys *or_keygen(const or_ctx *ctx, uint64_t seed, const int32_t *rots, int nrot);
void or_keys_free(or_keys *k);
/* secret key coefficients (ternary, N int64) */
const int64_t *or_keys_secret(const or_keys *k);
/* public key (b, a): [2][L+1][N] */
const uint64_t *or_keys_pk(const or_keys *k);
/* key-switching key for key id kid (Galois element, or 0 for s^2):
 * [dnum][2][L+1+nP][N] (b_t, a_t), NULL if absent */
const uint64_t *or_keys_ksk(const or_keys *k, uint64_t kid);

/* ---- encode / encrypt / decrypt / decode ---- */
/* Encode n <= N/2 real slot values (zero padded) at `level` with `scale`. */
or_pt *or_encode(const or_ctx *ctx, const double *z, int n, int level, double scale);
/* Same, always through the O(N^2) definition / always through the FFT. */
or_pt *or_encode_direct(const or_ctx *ctx, const double *z, int n, int level, double scale);
or_pt *or_encode_fft(const or_ctx *ctx, const double *z, int n, int level, double scale);
/* Integer plaintext from coefficient residues [level+1][N]. */
or_pt *or_pt_import(const or_ctx *ctx, const uint64_t *m, int level, double scale);
void or_pt_free(or_pt *p);
or_ct *or_encrypt(const or_ctx *ctx, const or_keys *k, const or_pt *p, uint64_t seed);
or_pt *or_decrypt(const or_ctx *ctx, const or_keys *k, const or_ct *ct);
/* Centered CRT lift of every coefficient to double (exact big-integer CRT). */
int or_pt_lift(const or_ctx *ctx, const or_pt *p, double *coeffs);
/* Decode the N/2 real slot values. */
int or_decode(const or_ctx *ctx, const or_pt *p, double *z);
int or_decode_direct(const or_ctx *ctx, const or_pt *p, double *z);
int or_decode_fft(const or_ctx *ctx, const or_pt *p, double *z);
or_ct *or_ct_import(const or_ctx *ctx, const uint64_t *c, int level, double scale);
or_ct *or_ct_copy(const or_ctx *ctx, const or_ct *a);
void or_ct_free(or_ct *c);

/* ---- homomorphic operations ---- */
/* out[i] = Rot_{rots[i]}(ct), sharing one ModUp of c1 (single hoisting). */
int or_rotate_hoisted(const or_ctx *ctx, const or_keys *k, const or_ct *ct,
                      const int32_t *rots, int nrot, or_ct **out);
or_ct *or_rescale(const or_ctx *ctx, const or_ct *a);
or_ct *or_add(const or_ctx *ctx, const or_ct *a, const or_ct *b);
or_ct *or_sub(const or_ctx *ctx, const or_ct *a, const or_ct *b);
or_ct *or_mul_plain(const or_ctx *ctx, const or_ct *a, const or_pt *p);
/* tensor, relinearise with the s^2 key, then rescale */
or_ct *or_mul_relin_rescale(const or_ctx *ctx, const or_keys *k, const or_ct *a, const or_ct *b);
/* sum of the tensor products of n pairs, relinearised once, rescaled */
or_ct *or_tensor_sum_relin_rescale(const or_ctx *ctx, const or_keys *k, const or_ct *const *a,
                                   const or_ct *const *b, int n);
/* P[0] + sum_{j >= 1} Rot_{j stride}(P[j]), the giant rotations sharing one
 * ModDown (inputs untouched) */
or_ct *or_rotate_sum(const or_ctx *ctx, const or_keys *k, const or_ct *const *P, int n, int stride);
/* multiply every limb by the signed integer kc (no rescale, scale *= kc) */
or_ct *or_mul_int(const or_ctx *ctx, const or_ct *a, int64_t kc);
/* add round(c * a->scale) to the constant coefficient of c0 */
or_ct *or_add_const(const or_ctx *ctx, const or_ct *a, double c);
or_ct *or_drop_to(const or_ctx *ctx, const or_ct *a, int level);

/* ---- database of pre-rotated plaintext diagonals ---- */
/* T: K rows of ell float32 values.  B blocks of ell x ell per plaintext,
 * n1 baby steps.  Diagonals encoded at `level` with scale `scale_d`. */
or_db *or_db_build(const or_ctx *ctx, const float *T, int K, int ell, int B, int n1,
                   int level, double scale_d);
/* Build from integer plaintexts: coeffs is [G][ell][level+1][N]. */
or_db *or_db_import(const or_ctx *ctx, const uint64_t *coeffs, int G, int ell, int B, int n1,
                    int level, double scale_d);
void or_db_free(or_db *db);
int or_db_groups(const or_db *db);
/* Export plaintext (group g, diagonal d) as coefficient residues [level+1][N]. */
int or_db_export(const or_db *db, int g, int d, uint64_t *out);
/* Residues of plaintext (g, d)'s centered integer coefficients modulo the
 * special primes, coefficient form [nP][N]. */
int or_db_export_special(const or_ctx *ctx, or_db *db, int g, int d, uint64_t *out);
/* Builds those residues for every diagonal now (else on the first hoisted product). */
int or_db_extend(const or_ctx *ctx, or_db *db);
/* Pre-rotated diagonal slot vector (group g, diagonal d) before encoding. */
int or_db_slots(const or_ctx *ctx, const float *T, int K, int ell, int B, int n1,
                int g, int d, double *v);
/* S_g = sum_j Rot_{j n1}( Rescale( sum_i baby[i] * diag'_{g, j n1 + i} ) ) */
or_ct *or_bsgs_matvec(const or_ctx *ctx, const or_keys *k, or_ct *const *baby, int n1,
                      const or_db *db, int group);
/* The same product from the query itself, with the baby steps kept over
 * Q_l U P (query and database at one level): with (a_j, b_j) =
 * sum_i B_i * diag'_{g, j n1 + i} over Q_l U P and B_i = Rot_i(ct) before
 * its ModDown, S_g = (Rescale(ModDown(sum_j sigma_{j n1}(a_j))),
 * Rescale(ModDown(b_0))) + sum_{j >= 1} KeySwitch_{j n1}(sigma_{j n1}(
 * Rescale(ModDown(b_j)))): the first polynomials, which rotate without a
 * key, take one ModDown together. */
or_ct *or_bsgs_matvec_hoisted(const or_ctx *ctx, const or_keys *k, const or_ct *x, int n1,
                              or_db *db, int group);

/* ---- Chebyshev threshold ---- */
/* Coefficients of the degree-n interpolant of the 0/1 step at delta on
 * [-1,1] through the n+1 first-kind Chebyshev nodes; c[0] is the full T_0
 * coefficient (p = sum_k c[k] T_k). */
void or_cheb_step_coeffs(int n, double delta, double *c);
/* Clenshaw evaluation of sum_k c[k] T_k(x) in FP64. */
double or_cheb_clenshaw(const double *c, int n, double x);
/* Homomorphic p(ct) by recursive Chebyshev-basis division with baby-step
 * degree d1. */
or_ct *or_chebyshev(const or_ctx *ctx, const or_keys *k, const or_ct *x,
                    const double *c, int n, int d1);
/* Count of relinearised products that or_chebyshev performs. */
int or_chebyshev_count_mults(int n, int d1);

#ifdef __cplusplus
}
#endif
#endif
