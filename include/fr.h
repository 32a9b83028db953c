/*
 * fr.h -- C ABI of the MI355X (gfx950) library for encrypted face-template
 * search: the RNS-CKKS baby-step giant-step diagonal matrix-vector product of
 * one encrypted query against a plaintext template database, followed by the
 * homomorphic Chebyshev threshold (arXiv 2604.00546).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Return value: FR_OK (0) or a negative fr_status; fr_last_error() then
 *   holds a thread-local message.  A failing call leaves its outputs' level
 *   and scale untouched and never frees caller memory.  Argument, level and
 *   key errors are found before any device work, so those outputs are not
 *   written at all; FR_ENOMEM (see fr_ctx_set_scratch_limit) can come after
 *   part of the work has run.
 * - Ring: R = Z[X]/(X^N + 1), N = 2^log_n.  Ciphertext modulus
 *   Q_l = q_0 ... q_l, special modulus P = p_0 ... p_{nP-1} (§3.2).
 * - fr_ct / fr_pt describe CALLER-OWNED device memory of uint64 words:
 *   a ciphertext at level l uses [2][l+1][N] words (c0 limbs, then c1 limbs),
 *   a plaintext [l+1][N].  `cap` is the largest level the buffer can hold
 *   (buffer size 2*(cap+1)*N resp. (cap+1)*N words); an output whose level
 *   would exceed `cap` is FR_EINVAL.  The words hold residues in the
 *   library's evaluation (NTT) form and order, which is private: use
 *   fr_ct_export / fr_pt_export for canonical coefficients.
 * - Keys and databases are LIBRARY-OWNED device objects (opaque handles),
 *   created by fr_keygen / fr_db_load / fr_db_import and freed by the
 *   matching destroy call.  They serve every context of the same parameter
 *   set on the same device (several contexts, each with its own stream and
 *   scratch, may use them at once; FR_EINVAL for another parameter set);
 *   they must outlive the work that uses them.
 * - Every device call is asynchronous on the context's stream (set with
 *   fr_ctx_set_stream; default: the null stream).  Calls that return data
 *   to the host (exports, fr_decode) synchronise that stream.  Inputs are
 *   never modified; an output may not alias an input unless stated.
 * - Host buffers for import/export hold COEFFICIENT form, natural order,
 *   canonical residues in [0, q_i), limb-major.
 */
#ifndef FR_H
#define FR_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fr_status {
    FR_OK = 0,
    FR_EINVAL = -1, /* bad argument, shape or capacity */
    FR_ENOMEM = -2, /* device allocation failed */
    FR_ELEVEL = -3, /* level or scale mismatch, or no level left */
    FR_ENOKEY = -4, /* a needed rotation / relinearisation key is absent */
    FR_EHIP = -5,   /* a HIP runtime call failed */
    FR_ERANGE = -6  /* a value does not fit the encoding (|coefficient| >= 2^62) */
} fr_status;

typedef struct fr_ctx fr_ctx;
typedef struct fr_keys fr_keys;
typedef struct fr_db fr_db;

/* Parameter set (§3.2; primes by the rule documented in the design notes:
 * q_0 = the largest q0_bits-bit prime = 1 mod 2N, q_1..q_L the next
 * largest mid_bits-bit primes in descending order, p_j the largest
 * special_bits-bit primes not already used).  Primes are at most 60 bits:
 * the base conversions and scalar combinations form exact sums of products
 * of 30-bit halves, which needs residues below 2^60. */
typedef struct fr_params {
    int32_t log_n;        /* 10 .. 16 */
    int32_t q0_bits;      /* 30 .. 60 */
    int32_t n_mid;        /* L: number of primes after q_0 */
    int32_t mid_bits;     /* 30 .. 60 */
    int32_t n_special;    /* number of special primes */
    int32_t special_bits; /* 30 .. 60 */
    int32_t dnum;         /* key-switching digits; alpha = ceil((L+1)/dnum) */
} fr_params;

typedef struct fr_ct {
    uint64_t *data; /* device, [2][level+1][N] */
    int32_t level;
    int32_t cap;
    double scale;
} fr_ct;

typedef struct fr_pt {
    uint64_t *data; /* device, [level+1][N] */
    int32_t level;
    int32_t cap;
    double scale;
} fr_pt;

const char *fr_last_error(void);

/* ---- context (setup of §3.2: primes, roots, RNS constants) ---- */
int fr_ctx_create(const fr_params *params, fr_ctx **out);
void fr_ctx_destroy(fr_ctx *ctx);
/* stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) */
int fr_ctx_set_stream(fr_ctx *ctx, void *stream);
int fr_ctx_sync(fr_ctx *ctx);
/* Device scratch (the memory term of Eq. stream-pool, §5.1.2).  Each context
 * keeps a growable device arena for the intermediate results of its calls
 * (ModUp digits, key inner products, inner sums, the Chebyshev ladder's
 * nodes); it grows on demand and is kept for later calls.
 * - fr_ctx_set_scratch_limit: the arena may total at most `bytes` (0: no
 *   limit).  If more is allocated now, the context waits for its streams and
 *   releases the arena.
 * - A call that needs more scratch than the limit (or than free device
 *   memory) returns FR_ENOMEM.  Its work already queued finishes before it
 *   returns; its outputs' level and scale are untouched, but the words of an
 *   output buffer may have been partly written.  The context stays usable.
 * - fr_ctx_scratch_info: bytes allocated now, and the most one call used.
 * - fr_ctx_reserve: grow the arena to at least `bytes` now (FR_ENOMEM if it
 *   cannot), so that later calls of that size allocate nothing. */
int fr_ctx_set_scratch_limit(fr_ctx *ctx, uint64_t bytes);
int fr_ctx_scratch_info(const fr_ctx *ctx, uint64_t *allocated, uint64_t *peak);
int fr_ctx_reserve(fr_ctx *ctx, uint64_t bytes);
/* Tuning knobs.  The project's autotuner sets them from measurements; every
 * value gives the same output words, only the kernel choice and the work per
 * launch change.
 * - FR_TUNE_NTT_{FWD_COLS4, FWD_ROWS4, INV_ROWS4, INV_COLS4}: the largest NTT
 *   launch (in limb polynomials) whose column / row pass at N = 2^16 takes 4
 *   words per thread in rounds of 2 stages (more threads, shorter chains)
 *   instead of 16 words per thread in rounds of 4 stages; 0 = never.
 * - FR_TUNE_MODUP_MERGE: inputs x digits up to which a ModUp runs as one
 *   conversion launch and one transform over every extended limb.
 * - FR_TUNE_MATVEC_CHUNK (1..16): queries per chunk of the batched products.
 * - FR_TUNE_CHEB_CHUNK (1..16): queries per pass of the batched Chebyshev
 *   evaluation.
 * - FR_TUNE_CHEB_SCHED (0 or 1): order of the Chebyshev evaluation's launch
 *   groups.  0: every node at its earliest depth, groups of a depth issued
 *   scalar family, products, additions.  1: level adjustments and scalar
 *   multiples at the latest depth before their first consumer, and the
 *   groups of a depth issued longest remaining path first.
 * - FR_TUNE_KSMAC (0..2): where the shape allows (n1 <= 32, ell = 16 n1, at
 *   most 3 digits), the hoisted product forms its baby steps inside the
 *   diagonal MAC (never written to memory): 0 never (a key inner product
 *   launch writes them and the MAC reads them), 1 for chunks of one query,
 *   2 for every chunk.
 * - FR_TUNE_KS_LDS (0 or 1): 1 = the giant steps' summed key inner products
 *   (at most 3 digits) copy each giant step's key slices into LDS one step
 *   ahead by wave-wide 16-byte loads; 0 = per-lane key loads.
 * FR_EINVAL for an unknown knob or a value out of range, and while a graph
 * capture is in progress. */
enum {
    FR_TUNE_NTT_FWD_COLS4 = 0,
    FR_TUNE_NTT_FWD_ROWS4 = 1,
    FR_TUNE_NTT_INV_ROWS4 = 2,
    FR_TUNE_NTT_INV_COLS4 = 3,
    FR_TUNE_MODUP_MERGE = 4,
    FR_TUNE_MATVEC_CHUNK = 5,
    FR_TUNE_CHEB_CHUNK = 6,
    FR_TUNE_CHEB_SCHED = 7,
    FR_TUNE_KSMAC = 8,
    FR_TUNE_KS_LDS = 9,
    FR_TUNE_COUNT = 10
};
int fr_ctx_set_tune(fr_ctx *ctx, int32_t knob, int32_t value);
int fr_ctx_get_tune(const fr_ctx *ctx, int32_t knob, int32_t *value);
/* N, L, nP, alpha, dnum */
int fr_ctx_dims(const fr_ctx *ctx, int32_t *n, int32_t *L, int32_t *n_special, int32_t *alpha,
                int32_t *dnum);
/* modulus by global index: 0..L = q_i, L+1 .. L+nP = p_j */
uint64_t fr_ctx_modulus(const fr_ctx *ctx, int32_t gidx);

/* ---- keys (§3.2 encryption; rotation keys of §4.2.3 / §5.3.2) ----
 * Secret key s uniform ternary, public key (b, a) = (-a s + e, a) mod Q_L,
 * one hybrid key-switching key per distinct Galois element 5^rot mod 2N of
 * `rots` (rotation 0 needs none) and one for s^2 (relinearisation).  All
 * randomness comes from Philox-4x64-10 keyed by `seed`. */
int fr_keygen(fr_ctx *ctx, uint64_t seed, const int32_t *rots, int32_t nrot, fr_keys **out);
void fr_keys_destroy(fr_keys *keys);
/* Export key material as canonical coefficients (test hook; synchronises).
 * what = 0: secret s as N int64 coefficients in {-1, 0, 1} (host_out is
 *           read as int64_t[N]);
 * what = 1: public key (b, a), [2][L+1][N];
 * what = 2: key-switching key for key id kid (Galois element, 0 = s^2),
 *           [dnum][2][L+1+nP][N] indexed by global modulus.
 * FR_ENOKEY if kid has no key. */
int fr_keys_export(fr_ctx *ctx, const fr_keys *keys, int32_t what, uint64_t kid, uint64_t *host_out);

/* ---- encode / encrypt / decrypt / decode (§3.2) ---- */
/* Encode n <= N/2 real slot values (host doubles, zero padded) at `level`
 * with `scale`: m_k = round(scale * (2/N) * sum_j z_j cos(pi 5^j k / N)),
 * computed by an FP64 FFT on the device. */
int fr_encode(fr_ctx *ctx, const double *z_host, int32_t n, int32_t level, double scale, fr_pt *out);
/* Same for a device slot vector (double, n entries). */
int fr_encode_device(fr_ctx *ctx, const double *z_dev, int32_t n, int32_t level, double scale,
                     fr_pt *out);
int fr_pt_import(fr_ctx *ctx, const uint64_t *coeff_host, int32_t level, double scale, fr_pt *out);
int fr_pt_export(fr_ctx *ctx, const fr_pt *pt, uint64_t *coeff_host);
/* ct = (v b + e0 + m, v a + e1) mod Q_l, v ternary, e0/e1 Gaussian from `seed`. */
int fr_encrypt(fr_ctx *ctx, const fr_keys *keys, const fr_pt *pt, uint64_t seed, fr_ct *out);
/* m = c0 + c1 s mod Q_l */
int fr_decrypt(fr_ctx *ctx, const fr_keys *keys, const fr_ct *ct, fr_pt *out);
/* Centered CRT lift and forward canonical embedding: n <= N/2 slot values
 * z_j = Re m(zeta^(5^j)) / scale.  Requires |m_k| < 2^62 (FR_ERANGE). */
int fr_decode(fr_ctx *ctx, const fr_pt *pt, double *z_host, int32_t n);
int fr_ct_import(fr_ctx *ctx, const uint64_t *coeff_host, int32_t level, double scale, fr_ct *out);
int fr_ct_export(fr_ctx *ctx, const fr_ct *ct, uint64_t *coeff_host);

/* ---- homomorphic operations ---- */
/* Single-hoisted rotations (§3.4.2): outs[i] = Rot_{rots[i]}(in), a left
 * slot rotation, for every i, sharing one ModUp of c1.  Each Rot is
 * (sigma_g(c0) + ModDown(U0), ModDown(U1)) with U = sum_t sigma_g(ModUp_t(c1))
 * * ksk_{g,t}.  outs must not alias in.  FR_ENOKEY if a key is absent. */
int fr_rotate_hoisted(fr_ctx *ctx, const fr_keys *keys, const fr_ct *in, const int32_t *rots,
                      int32_t nrot, fr_ct *outs);
/* Batched form (queries sharing the rotation keys, the served setting of
 * §5.1.2 where many matrices and queries are in flight): in[0..nq-1] at one
 * level, outs[q * nrot + r] = Rot_{rots[r]}(in[q]).  Each query's outputs are
 * the words fr_rotate_hoisted returns for it alone; each key is read once
 * per rotation for the whole batch.  No output may alias any input. */
int fr_rotate_hoisted_batch(fr_ctx *ctx, const fr_keys *keys, const fr_ct *in, int32_t nq,
                            const int32_t *rots, int32_t nrot, fr_ct *outs);
/* Allocation-free form of fr_rotate_hoisted, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results (the same words)
 * and errors as fr_rotate_hoisted; it calls no hipMalloc, hipFree or other
 * allocating routine.  Its scratch (the ModUp digits, the key inner products
 * and the ModDown corrections) is a fixed device array of
 * FR_NOALLOC_SCRATCH_BYTES per GPU, created with the library's code object
 * and held until the process ends; rotations are taken in chunks that fit
 * in it.  FR_ENOMEM, before any device work, when one rotation of `in`
 * needs more than the array (at N = 2^16 a rotation needs 77.5 MiB at 15 Q
 * limbs and 5 special primes, dnum 3).  Every call on one GPU, from any
 * context or stream, uses the same array and leaves its contents behind:
 * calls that overlap on one GPU race and must be ordered by the caller. */
#define FR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int fr_rotate_hoisted_noalloc(fr_ctx *ctx, const fr_keys *keys, const fr_ct *in, const int32_t *rots,
                              int32_t nrot, fr_ct *outs);
/* Rescale (§3.2): drop q_l with centered rounding; scale /= q_l. */
int fr_rescale(fr_ctx *ctx, const fr_ct *in, fr_ct *out);
int fr_add(fr_ctx *ctx, const fr_ct *a, const fr_ct *b, fr_ct *out);
int fr_sub(fr_ctx *ctx, const fr_ct *a, const fr_ct *b, fr_ct *out);
/* plaintext x ciphertext product (no rescale); scale multiplies */
int fr_mul_plain(fr_ctx *ctx, const fr_ct *a, const fr_pt *p, fr_ct *out);
/* ciphertext x ciphertext: tensor, relinearise with the s^2 key, rescale */
int fr_mul_relin_rescale(fr_ctx *ctx, const fr_keys *keys, const fr_ct *a, const fr_ct *b, fr_ct *out);
/* multiply by a signed integer (scale *= k) / add round(c * scale) / drop limbs */
int fr_mul_int(fr_ctx *ctx, const fr_ct *a, int64_t k, fr_ct *out);
int fr_add_const(fr_ctx *ctx, const fr_ct *a, double c, fr_ct *out);
int fr_drop_to(fr_ctx *ctx, const fr_ct *a, int32_t level, fr_ct *out);

/* ---- database of pre-rotated plaintext diagonals (§3.3.1 packing,
 * Eq. diag, Eq. prerotation of §5.3.1 applied in the slot domain by the
 * enroller as in §5.3.3) ----
 * T_host: K rows of ell float32 values (unit-norm templates).  B blocks of
 * ell x ell per plaintext (B * ell <= N/2), G = ceil(K / (B ell)) groups of ell
 * plaintexts, n1 baby steps.  Diagonal d = j n1 + i of group g is the slot
 * vector diag_d[b ell + r] = T[(g B + b) ell + r][(r + d) mod ell], rotated
 * left by -j n1 over all N/2 slots, encoded at `level` with `scale`, kept
 * resident in HBM. */
int fr_db_load(fr_ctx *ctx, const float *T_host, int32_t K, int32_t ell, int32_t B, int32_t n1,
               int32_t level, double scale, fr_db **out);
/* The same from integer plaintexts [G][ell][level+1][N] (coefficient form). */
int fr_db_import(fr_ctx *ctx, const uint64_t *coeff_host, int32_t G, int32_t ell, int32_t B,
                 int32_t n1, int32_t level, double scale, fr_db **out);
int fr_db_export(fr_ctx *ctx, const fr_db *db, int32_t group, int32_t diag, uint64_t *coeff_host);
int fr_db_groups(const fr_db *db);
void fr_db_destroy(fr_db *db);

/* ---- the hot path (Eq. bsgs2 of §3.4, Alg. gpu-bsgs-index of §5.4) ----
 * baby[i] = Rot_i(query), i < n1 (baby[0] = query), all at one level and
 * scale.  For group g:
 *   P_j = Rescale( sum_{i < min(n1, ell - j n1)} baby[i] * diag'_{g, j n1 + i} )
 *   out = P_0 + sum_{j >= 1} Rot_{j n1}(P_j),
 * the giant rotations sharing one ModDown.  Slot s of out is the score of
 * template g B ell + s. */
int fr_bsgs_diag_matvec(fr_ctx *ctx, const fr_keys *keys, const fr_ct *baby, int32_t n1,
                        const fr_db *db, int32_t group, fr_ct *out);
/* Batched form: baby[q * n1 + i] is baby step i of query q (every query's
 * steps at one level), scored against group groups[q] of dbs[q] (databases
 * of one ell, n1 and level; sizes may differ); out[q] is its score
 * ciphertext, identical to the one-query call.  Queries are ordered by
 * diagonal group and processed in chunks of up to 8: each chunk reads every
 * diagonal of each of its groups and every giant-step key once. */
int fr_bsgs_diag_matvec_batch(fr_ctx *ctx, const fr_keys *keys, const fr_ct *baby, int32_t nq,
                              int32_t n1, const fr_db *const *dbs, const int32_t *groups, fr_ct *out);

/* ---- the same product with the baby steps' ModDown hoisted past the inner
 * sums (double hoisting of the plaintext-matrix BSGS, §3.4.2 hoisting and double
 * hoisting) ----
 * fr_db_extend appends to every diagonal of db its residues modulo the
 * special primes (those of the plaintext's centered integer coefficients,
 * exact), growing the database by nP / (level+1).  Idempotent; the
 * database stays valid for every other call.  FR_ENOMEM leaves it as it was.
 *
 * fr_bsgs_matvec_hoisted computes the score ciphertext from the query
 * itself (query level = database level = l >= 1, n1 = the database's):
 *   B_0 = (P c0, P c1),  B_i = (P sigma_i(c0) + U0_i, U1_i) over Q_l U P,
 *   U_i = sum_t sigma_i(ModUp_t(c1)) ksk_{i,t}   (Rot_i before its ModDown),
 *   (a_j, b_j) = sum_i B_i * diag'_{g, j n1 + i}   over Q_l U P,
 *   out = (Rescale(ModDown(sum_j sigma_{j n1}(a_j))), Rescale(ModDown(b_0)))
 *         + sum_{j >= 1} KeySwitch_{j n1}(sigma_{j n1}(Rescale(ModDown(b_j))))
 * at level l-1 (the key switches sharing one ModDown; a rotation needs no
 * key for the first polynomials, which are summed before their ModDown),
 * keys for rotations 1..n1-1 and j n1.  The scores approximate those of
 * fr_rotate_hoisted + fr_bsgs_diag_matvec with one ModDown per inner sum
 * instead of one per baby step; the words differ (other rounding).
 * FR_EINVAL for a database that is not extended. */
int fr_db_extend(fr_ctx *ctx, fr_db *db);
int fr_bsgs_matvec_hoisted(fr_ctx *ctx, const fr_keys *keys, const fr_ct *query, const fr_db *db,
                           int32_t group, fr_ct *out);
/* Batched form: query q against group groups[q] of dbs[q] (extended, one
 * ell, n1 and level); out[q] identical to the one-query call; chunks of up
 * to 8 queries read every diagonal and key once per chunk. */
int fr_bsgs_matvec_hoisted_batch(fr_ctx *ctx, const fr_keys *keys, const fr_ct *queries, int32_t nq,
                                 const fr_db *const *dbs, const int32_t *groups, fr_ct *out);

/* ---- Chebyshev threshold (§5.1.4, Eq. cheb-sign) ----
 * out = p(in) slot-wise, p = sum_{k <= degree} c[k] T_k (c[0] the full T_0
 * coefficient), evaluated by recursive Chebyshev-basis division over
 * baby-step powers T_1..T_{d1-1} and giant powers T_{d1 2^j}, with
 * canonical per-level scales (reading documented in the design notes). */
int fr_chebyshev_eval(fr_ctx *ctx, const fr_keys *keys, const fr_ct *in, const double *c,
                      int32_t degree, int32_t d1, fr_ct *out);
/* Batched form: out[q] = p(in[q]) for nq inputs of one level and scale,
 * identical to nq calls of fr_chebyshev_eval; every wave of the evaluation
 * runs for up to 8 queries at once. */
int fr_chebyshev_eval_batch(fr_ctx *ctx, const fr_keys *keys, const fr_ct *in, int32_t nq,
                            const double *c, int32_t degree, int32_t d1, fr_ct *out);

/* ---- encrypted-database product (§3.3.1 encrypts the diagonal rows; the
 * relinearisation is deferred to one per sum, §3.4.1) ----
 * out = Rescale(Relin(sum_k a[k] (x) b[k])): the tensor products (a0 b0,
 * a0 b1 + a1 b0, a1 b1) of the n pairs are summed as one degree-2
 * ciphertext, relinearised once with the s^2 key and rescaled.  With a[k] the
 * query rotations and b[k] the encrypted diagonals of a group this is the
 * group's score ciphertext.  All 2n inputs at one level >= 1 and every
 * product at one scale; out->level = level - 1.  FR_ENOKEY without the
 * relinearisation key. */
int fr_tensor_sum_relin_rescale(fr_ctx *ctx, const fr_keys *keys, const fr_ct *a, const fr_ct *b, int32_t n,
                                fr_ct *out);

/* ---- giant-step rotate-sum (Eq. bsgs2 of §3.4; the on-demand giant
 * rotations of §5.3.2) ----
 * out = in[0] + sum_{j >= 1} Rot_{j stride}(in[j]): the n inputs (one level
 * and scale) are rotated by their giant steps, the key inner products summed
 * over Q_l U P and taken through one shared ModDown.  Keys for the rotations
 * j stride; out at the inputs' level; out must not alias an input. */
int fr_rotate_sum(fr_ctx *ctx, const fr_keys *keys, const fr_ct *in, int32_t n, int32_t stride, fr_ct *out);

/* ---- BSGS product against an encrypted database (BSGS-TBS / TBE of
 * §5.3: pre-rotated encrypted diagonals, Eq. prerotation of §5.3.1; the
 * online pipeline of §5.3.2 with lazy relinearisation per giant step) ----
 * baby[i] = Rot_i(query), i < n1; diag[d], d < ell, the group's encrypted
 * diagonals pre-rotated by -j n1 (d = j n1 + i) -- homomorphically by the
 * server with temporary negative giant-step keys (TBS: fr_rotate_hoisted_batch
 * with rotation -j n1 on the diagonals of giant step j) or in the plaintext
 * slots by the enroller before encryption (TBE); all at one level l >= 1.
 *   P_j = Rescale(Relin(sum_{i < min(n1, ell - j n1)} baby[i] (x) diag[j n1 + i]))
 *   out = P_0 + sum_{j >= 1} Rot_{j n1}(P_j)   (level l-1)
 * The tensor sums are degree 2 and relinearised once per giant step; the
 * giant rotations share one ModDown.  Needs the s^2 key and the keys for
 * j n1.  Slot s of out is the score of the group's template s. */
int fr_bsgs_encrypted_matvec(fr_ctx *ctx, const fr_keys *keys, const fr_ct *baby, int32_t n1, const fr_ct *diag,
                             int32_t ell, fr_ct *out);

/* ---- membership aggregation (Alg. gpu-bsgs-membership, aggregation step;
 * Alg. membership of the appendix: EvalAddMany then EvalSum over all slots) ----
 * out = EvalSum(in[0] + ... + in[n-1]): the n inputs (one level and scale,
 * typically the Chebyshev outputs of every group) are added, then log2(N/2)
 * doublings x <- x + Rot_{2^i}(x) put the sum of all N/2 slots in every slot
 * (slot 0 = the number of templates over the threshold).  Needs the rotation
 * keys 2^i, i < log2(N/2) (FR_ENOKEY otherwise).  out must not alias any
 * input; out->level = in[0].level. */
int fr_membership_aggregate(fr_ctx *ctx, const fr_keys *keys, const fr_ct *in, int32_t n, fr_ct *out);

/* ---- captured call sequences (HIP graphs; the per-query launch sequence of
 * Alg. gpu-bsgs-index replayed as one graph) ----
 * fr_graph_begin: the device calls made on ctx until fr_graph_end are
 *   recorded, not run (stream capture of a private stream of the context and
 *   of its auxiliary streams; the caller's stream is waited for first).
 *   Only calls that need no host result may be recorded: rotations, the
 *   products, rescale, add/sub, the Chebyshev evaluation, membership
 *   aggregation, encryption.  A call that synchronises (exports, imports,
 *   decode, key or database setup, the timing hook) makes fr_graph_end fail.
 * fr_graph_end: ends the recording and instantiates the graph (*out, freed
 *   with fr_graph_destroy).  FR_EHIP if the capture was broken.
 * fr_graph_launch: replays the graph on the context's stream.  The kernels
 *   read and write the device addresses of the recording: the callers'
 *   buffers and the context's scratch, so new data is given by writing it
 *   into the recorded input buffers before the launch.  Replays and other
 *   calls of the context are ordered on its stream.  FR_EINVAL if the
 *   context's scratch was released since the recording
 *   (fr_ctx_set_scratch_limit below the allocation). */
/* Switched off: fr_graph_begin returns FR_EINVAL.  A recording of the
 * hoisted product followed by the Chebyshev ladder ended in a host fault
 * inside the HIP runtime's capture end, with no cause established; the
 * calls stay declared so that callers compile unchanged. */
typedef struct fr_graph fr_graph;
int fr_graph_begin(fr_ctx *ctx);
int fr_graph_end(fr_ctx *ctx, fr_graph **out);
int fr_graph_launch(fr_ctx *ctx, const fr_graph *graph);
void fr_graph_destroy(fr_graph *graph);

/* ---- parity hook: ModDown on caller-given residues (hybrid key switching
 * of §3.4.2; the rescale of §3.2) ----
 * u_host: [2][level+1+nP][N] canonical coefficient-form residues over
 * Q_level U P (limbs q_0..q_level, then p_0..p_{nP-1}); d_host (mode 2
 * only): [2][level+1][N] over Q_level.  ModDown(u) = round(u / P)
 * coefficient-wise (u minus its centered residue mod P, divided by P), with
 * the rounding decided exactly.  The result runs through the same device
 * path as the hot path's ModDown of that kind:
 *   mode 0: out = ModDown(u) at `level` (key switching of a rotation);
 *   mode 1: out = Rescale(ModDown(u)) at level-1 (the inner sums of
 *           fr_bsgs_matvec_hoisted);
 *   mode 2: out = Rescale(d + ModDown(u)) at level-1 (a relinearised
 *           product).
 * out->scale is set to 1.  Synchronises.  FR_EINVAL for a residue that is
 * not canonical; FR_ELEVEL for level < 1 in modes 1 and 2. */
int fr_moddown_parity(fr_ctx *ctx, int32_t mode, const uint64_t *u_host, const uint64_t *d_host, int32_t level,
                      fr_ct *out);

/* ---- kernel timing hook (for the benchmark's roofline figures) ----
 * While a class is selected, every launch of that kernel class is bracketed
 * by HIP events on the context's stream and its algorithmic HBM bytes (the
 * words the operation must read and write once) are added up.  Classes:
 * 1 NTT (one forward or inverse transform of a batch of limbs), 2 ModUp base
 * conversion, 3 key-switching inner product, 4 ModDown base conversion,
 * 5 plaintext-diagonal multiply-accumulate, 6 rescale, 7 tensor product,
 * 8 element-wise arithmetic.  fr_prof_end synchronises, returns the launch
 * count, summed event time (ms) and bytes, and deselects the class. */
int fr_prof_begin(fr_ctx *ctx, int32_t kernel_class);
int fr_prof_end(fr_ctx *ctx, int32_t *launches, double *total_ms, double *bytes);

/* ---- host-only planning helpers (no device work) ---- */
/* degree-n interpolant of the 0/1 step at delta through the n+1 first-kind
 * Chebyshev nodes ("DCT-based interpolation" of §5.1.4); c[0] full T_0. */
int fr_cheb_step_coeffs(int32_t degree, double delta, double *c);
/* Paterson-Stockmeyer split of §5.1.4: minimise d1 + d2 subject to
 * d1 2^(d2-1) >= degree, d1 >= 2, ties to the smaller d1. */
int fr_cheb_ps_params(int32_t degree, int32_t *d1, int32_t *d2);
/* Output level of fr_chebyshev_eval for an input at in_level (-1 if the
 * levels run out); number of relinearised products it performs. */
int fr_cheb_out_level(int32_t in_level, int32_t degree, int32_t d1);
int fr_cheb_mult_count(int32_t degree, int32_t d1);
/* Eq. stream-pool of §5.1.2: S = min(floor(units/4), floor(0.2 F / (40 C)), 32), S >= 2. */
int fr_stream_pool_size(int32_t compute_units, double free_bytes, double ct_bytes);
/* Rotation-key index set of §4.2.3: S_baby = {1..n1-1}, S_giant = {j n1 : 1 <= j < n2},
 * n2 = ceil(ell / n1).  Writes up to cap indices, returns the count. */
int fr_bsgs_rotation_set(int32_t ell, int32_t n1, int32_t *out, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif
