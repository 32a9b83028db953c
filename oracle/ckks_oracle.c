/*
 * ckks_oracle.c -- plain, slow, obviously-correct CPU oracle of the paper's
 * hot path (arXiv 2604.00546): RNS-CKKS (§3.2), the diagonal method (Eq. diag,
 * §3.3), its grouped baby-step giant-step form (Eq. bsgs2, §3.4) with
 * pre-rotated plaintext diagonals (Eq. prerotation, §5.3.1 and the
 * enroller-side variant of §5.3.3), single hoisting of the baby-step rotations
 * (§3.4.2), and the Chebyshev threshold of §5.1.4.
 *
 * TEST INFRASTRUCTURE ONLY -- see ckks_oracle.h.  Shares nothing with the HIP
 * library.  Where the paper is silent the reading taken is written next to the
 * code that implements it; the same readings are listed in the design notes.
 *
 * Build: gcc -O2 -std=gnu11 -fopenmp -ffp-contract=off -fPIC -shared
 */
#include "ckks_oracle.h"

#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define OR_MAXMOD 64

static __thread char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *or_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* modular arithmetic, written out with 128-bit products and remainders      */
/* ------------------------------------------------------------------------ */
static inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * b) % q);
}
static inline uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    uint64_t s = a + b; /* a, b < q < 2^62: no wrap */
    return s >= q ? s - q : s;
}
static inline uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
    return a >= b ? a - b : a + (q - b);
}
static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); } /* q prime */
static uint64_t smod(int64_t v, uint64_t q) {
    if (v >= 0) return (uint64_t)v % q;
    uint64_t r = (uint64_t)(-(v + 1)) % q; /* -(v+1) avoids overflow at INT64_MIN */
    r = (r + 1) % q;
    return r == 0 ? 0 : q - r;
}

/* Deterministic Miller-Rabin; the first twelve prime bases decide every
 * n < 3.3e24, so every 64-bit n. */
static int is_prime_u64(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n % bases[i] == 0) return n == bases[i];
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

static int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* ------------------------------------------------------------------------ */
/* exact CRT lift with little multi-word integers                            */
/* ------------------------------------------------------------------------ */
#define BW 40 /* words: enough for 40 primes of < 64 bits */
typedef struct { uint64_t w[BW]; } big;
static void big_zero(big *a) { memset(a, 0, sizeof *a); }
static void big_mul_small(big *a, uint64_t m) {
    u128 carry = 0;
    for (int i = 0; i < BW; i++) {
        u128 t = (u128)a->w[i] * m + carry;
        a->w[i] = (uint64_t)t;
        carry = t >> 64;
    }
}
static void big_add(big *a, const big *b) {
    u128 carry = 0;
    for (int i = 0; i < BW; i++) {
        u128 t = (u128)a->w[i] + b->w[i] + carry;
        a->w[i] = (uint64_t)t;
        carry = t >> 64;
    }
}
static void big_sub(big *a, const big *b) { /* a >= b */
    uint64_t borrow = 0;
    for (int i = 0; i < BW; i++) {
        uint64_t bi = b->w[i], ai = a->w[i];
        uint64_t d = ai - bi - borrow;
        borrow = (ai < bi) || (ai - bi < borrow);
        a->w[i] = d;
    }
}
static int big_cmp(const big *a, const big *b) {
    for (int i = BW - 1; i >= 0; i--) {
        if (a->w[i] != b->w[i]) return a->w[i] > b->w[i] ? 1 : -1;
    }
    return 0;
}
static double big_to_double(const big *a) {
    double r = 0.0;
    for (int i = BW - 1; i >= 0; i--) r = r * 18446744073709551616.0 + (double)a->w[i];
    return r;
}

/* ------------------------------------------------------------------------ */
/* context                                                                    */
/* ------------------------------------------------------------------------ */
struct or_ctx {
    int logN, N, L, nP, dnum, alpha;
    int nmod;
    uint64_t mod[OR_MAXMOD];
    uint64_t psi[OR_MAXMOD];
    uint64_t *psi_pow[OR_MAXMOD];  /* psi^k, k < N */
    uint64_t *psi_ipow[OR_MAXMOD]; /* psi^-k * N^-1, k < N */
    uint64_t *w_pow[OR_MAXMOD];    /* omega^k, omega = psi^2, k < N/2 */
    uint64_t *w_ipow[OR_MAXMOD];   /* omega^-k, k < N/2 */
    uint64_t cdt[20];
    double *costab;   /* cos(pi t / N), t < 2N */
    uint64_t *pow5;   /* 5^j mod 2N, j < N/2 */
};

int or_ctx_N(const or_ctx *c) { return c->N; }
int or_ctx_L(const or_ctx *c) { return c->L; }
int or_ctx_nspecial(const or_ctx *c) { return c->nP; }
int or_ctx_alpha(const or_ctx *c) { return c->alpha; }
uint64_t or_ctx_modulus(const or_ctx *c, int g) { return (g >= 0 && g < c->nmod) ? c->mod[g] : 0; }

/* Walk down from 2^bits through the candidates c = 1 mod 2N below 2^bits and
 * return the first prime that is not in `used`.  Reading of the parameter
 * rule: a "b-bit prime" is a prime below 2^b (and at or above 2^(b-1)); the
 * chain takes the largest such primes, in descending order. */
static uint64_t next_prime_below(uint64_t *cursor, uint64_t twoN, const uint64_t *used, int nused) {
    for (;;) {
        uint64_t c = *cursor;
        *cursor -= twoN;
        if (!is_prime_u64(c)) continue;
        int dup = 0;
        for (int i = 0; i < nused; i++) dup |= (used[i] == c);
        if (!dup) return c;
    }
}

or_ctx *or_ctx_create(int logN, int q0_bits, int n_mid, int mid_bits,
                      int n_special, int special_bits, int dnum) {
    if (logN < 3 || logN > 17 || q0_bits < 20 || q0_bits > 61 || mid_bits < 20 || mid_bits > 61 ||
        special_bits < 20 || special_bits > 61 || n_mid < 0 || n_special < 1 || dnum < 1 ||
        1 + n_mid + n_special > OR_MAXMOD) {
        set_err("or_ctx_create: parameter out of range");
        return NULL;
    }
    or_ctx *c = calloc(1, sizeof *c);
    c->logN = logN;
    c->N = 1 << logN;
    c->L = n_mid;
    c->nP = n_special;
    c->dnum = dnum;
    c->alpha = (c->L + 1 + dnum - 1) / dnum;
    c->nmod = c->L + 1 + c->nP;
    const uint64_t twoN = 2ull * (uint64_t)c->N;
    uint64_t used[OR_MAXMOD] = {0};
    int nused = 0;
    /* q_0: the largest q0_bits-bit prime = 1 mod 2N */
    uint64_t cur = (1ull << q0_bits) - twoN + 1;
    c->mod[0] = next_prime_below(&cur, twoN, used, nused);
    used[nused++] = c->mod[0];
    /* q_1..q_L: the largest mid_bits-bit primes, descending */
    uint64_t cur_mid = (1ull << mid_bits) - twoN + 1;
    for (int i = 1; i <= c->L; i++) {
        c->mod[i] = next_prime_below(&cur_mid, twoN, used, nused);
        used[nused++] = c->mod[i];
    }
    /* p_0..p_{nP-1}: the largest special_bits-bit primes not used above */
    uint64_t cur_sp = (1ull << special_bits) - twoN + 1;
    for (int j = 0; j < c->nP; j++) {
        c->mod[c->L + 1 + j] = next_prime_below(&cur_sp, twoN, used, nused);
        used[nused++] = c->mod[c->L + 1 + j];
    }
    const int N = c->N;
    for (int m = 0; m < c->nmod; m++) {
        uint64_t q = c->mod[m];
        /* a primitive 2N-th root of unity: x^((q-1)/2N) with psi^N = -1 */
        uint64_t psi = 0;
        for (uint64_t x = 2;; x++) {
            psi = powmod(x, (q - 1) / twoN, q);
            if (powmod(psi, (uint64_t)N, q) == q - 1) break;
        }
        c->psi[m] = psi;
        uint64_t psi_inv = invmod(psi, q), ninv = invmod((uint64_t)N, q);
        uint64_t omega = mulmod(psi, psi, q), omega_inv = invmod(omega, q);
        c->psi_pow[m] = malloc(sizeof(uint64_t) * N);
        c->psi_ipow[m] = malloc(sizeof(uint64_t) * N);
        c->w_pow[m] = malloc(sizeof(uint64_t) * (N / 2));
        c->w_ipow[m] = malloc(sizeof(uint64_t) * (N / 2));
        uint64_t a = 1, b = ninv;
        for (int k = 0; k < N; k++) {
            c->psi_pow[m][k] = a;
            c->psi_ipow[m][k] = b;
            a = mulmod(a, psi, q);
            b = mulmod(b, psi_inv, q);
        }
        a = 1; b = 1;
        for (int k = 0; k < N / 2; k++) {
            c->w_pow[m][k] = a;
            c->w_ipow[m][k] = b;
            a = mulmod(a, omega, q);
            b = mulmod(b, omega_inv, q);
        }
    }
    or_gauss_cdt(c->cdt);
    c->costab = malloc(sizeof(double) * 2 * N);
    for (int t = 0; t < 2 * N; t++) c->costab[t] = cos(M_PI * (double)t / (double)N);
    c->pow5 = malloc(sizeof(uint64_t) * (N / 2));
    uint64_t e = 1;
    for (int j = 0; j < N / 2; j++) { c->pow5[j] = e; e = (e * 5) % twoN; }
    return c;
}

void or_ctx_free(or_ctx *c) {
    if (!c) return;
    for (int m = 0; m < c->nmod; m++) {
        free(c->psi_pow[m]); free(c->psi_ipow[m]); free(c->w_pow[m]); free(c->w_ipow[m]);
    }
    free(c->costab);
    free(c->pow5);
    free(c);
}

/* Galois element of a left rotation by `rot` slots: 5^rot mod 2N, with a
 * negative rotation taken as rot mod N/2 (5 has order N/2 mod 2N). §3.2
 * rotation paragraph; the slot order is the 5^j order of the encoding. */
uint64_t or_galois_element(const or_ctx *c, int rot) {
    int h = c->N / 2;
    int r = ((rot % h) + h) % h;
    return c->pow5[r];
}

/* ------------------------------------------------------------------------ */
/* textbook negacyclic NTT: twist by psi^k, cyclic radix-2 DIT NTT with      */
/* omega = psi^2 (bit-reversal permutation first), and back.                 */
/* ------------------------------------------------------------------------ */
static void ntt_cyclic(uint64_t *a, int N, int logN, const uint64_t *wpow, uint64_t q) {
    for (int i = 0; i < N; i++) {
        int j = bitrev(i, logN);
        if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= N; len <<= 1) {
        int half = len >> 1, step = N / len;
        for (int i = 0; i < N; i += len) {
            for (int j = 0; j < half; j++) {
                uint64_t u = a[i + j];
                uint64_t v = mulmod(a[i + j + half], wpow[j * step], q);
                a[i + j] = addmod(u, v, q);
                a[i + j + half] = submod(u, v, q);
            }
        }
    }
}
/* forward: coefficients -> values at psi^(2k+1) (in the cyclic NTT's order) */
static void nega_fwd(const or_ctx *c, int m, uint64_t *a) {
    uint64_t q = c->mod[m];
    for (int k = 0; k < c->N; k++) a[k] = mulmod(a[k], c->psi_pow[m][k], q);
    ntt_cyclic(a, c->N, c->logN, c->w_pow[m], q);
}
static void nega_inv(const or_ctx *c, int m, uint64_t *a) {
    uint64_t q = c->mod[m];
    ntt_cyclic(a, c->N, c->logN, c->w_ipow[m], q);
    for (int k = 0; k < c->N; k++) a[k] = mulmod(a[k], c->psi_ipow[m][k], q);
}

int or_polymul(const or_ctx *c, int m, const uint64_t *a, const uint64_t *b, uint64_t *out) {
    if (m < 0 || m >= c->nmod) { set_err("or_polymul: bad modulus index"); return -1; }
    int N = c->N;
    uint64_t q = c->mod[m];
    uint64_t *ta = malloc(8 * (size_t)N), *tb = malloc(8 * (size_t)N);
    memcpy(ta, a, 8 * (size_t)N);
    memcpy(tb, b, 8 * (size_t)N);
    nega_fwd(c, m, ta);
    nega_fwd(c, m, tb);
    for (int k = 0; k < N; k++) ta[k] = mulmod(ta[k], tb[k], q);
    nega_inv(c, m, ta);
    memcpy(out, ta, 8 * (size_t)N);
    free(ta); free(tb);
    return 0;
}

/* sigma_g: X^i -> X^(i g mod 2N), with X^N = -1 (coefficient domain). */
void or_automorphism(const or_ctx *c, int m, uint64_t g, const uint64_t *a, uint64_t *out) {
    int N = c->N;
    uint64_t q = c->mod[m], twoN = 2ull * (uint64_t)N;
    for (int i = 0; i < N; i++) {
        uint64_t e = ((uint64_t)i * g) % twoN;
        if (e < (uint64_t)N) out[e] = a[i];
        else out[e - N] = a[i] ? q - a[i] : 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Philox-4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11) and the samplers built on it.                     */
/* ------------------------------------------------------------------------ */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += W0; k1 += W1; }
        u128 p0 = (u128)M0 * x0, p1 = (u128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One Philox block of the stream (seed, domain): counter (idx, limb, poly, 0),
 * key (seed, domain).  Domains: 1 uniform, 2 ternary, 3 Gaussian. */
static void rng_block(uint64_t seed, uint64_t dom, uint64_t poly, uint64_t limb, uint64_t idx,
                      uint64_t out[4]) {
    uint64_t ctr[4] = {idx, limb, poly, 0}, key[2] = {seed, dom};
    or_philox4x64_10(ctr, key, out);
}

/* Cumulative table of |e| for the discrete Gaussian rho(x) = exp(-x^2/(2 sigma^2)),
 * sigma = 3.2, tail cut at |x| <= 19, scaled to 2^63.  The exact FP64
 * expression order is part of the definition. */
void or_gauss_cdt(uint64_t cdt[20]) {
    double rho[20];
    for (int t = 0; t < 20; t++) rho[t] = exp(-(double)(t * t) / (2.0 * 3.2 * 3.2));
    double S = rho[0];
    for (int t = 1; t < 20; t++) S += 2.0 * rho[t];
    double cum = 0.0;
    for (int t = 0; t < 20; t++) {
        cum += (t == 0 ? rho[0] : 2.0 * rho[t]) / S;
        cdt[t] = (t == 19) ? (1ull << 63) : (uint64_t)ldexp(cum, 63);
    }
}

/* Uniform residue mod q of coefficient k of global limb gidx: the 128-bit
 * integer (hi, lo) taken from half a Philox block, reduced mod q. */
void or_sample_uniform(uint64_t seed, uint64_t poly, int gidx, uint64_t q, int N, uint64_t *out) {
    for (int b = 0; b < N / 2; b++) {
        uint64_t r[4];
        rng_block(seed, 1, poly, (uint64_t)gidx, (uint64_t)b, r);
        for (int u = 0; u < 2; u++) {
            u128 v = ((u128)r[2 * u + 1] << 64) | r[2 * u];
            out[2 * b + u] = (uint64_t)(v % q);
        }
    }
}
/* Uniform ternary coefficient: (word mod 3) - 1. */
void or_sample_ternary(uint64_t seed, uint64_t poly, int N, int64_t *out) {
    for (int b = 0; b < N / 4; b++) {
        uint64_t r[4];
        rng_block(seed, 2, poly, 0, (uint64_t)b, r);
        for (int u = 0; u < 4; u++) out[4 * b + u] = (int64_t)(r[u] % 3) - 1;
    }
}
/* Discrete Gaussian: top bit = sign, low 63 bits looked up in the CDT. */
void or_sample_gauss(uint64_t seed, uint64_t poly, int N, int64_t *out) {
    uint64_t cdt[20];
    or_gauss_cdt(cdt);
    for (int b = 0; b < N / 4; b++) {
        uint64_t r[4];
        rng_block(seed, 3, poly, 0, (uint64_t)b, r);
        for (int u = 0; u < 4; u++) {
            uint64_t sign = r[u] >> 63, v = r[u] & 0x7FFFFFFFFFFFFFFFull;
            int t = 0;
            while (v >= cdt[t]) t++;
            out[4 * b + u] = (sign && t) ? -(int64_t)t : (int64_t)t;
        }
    }
}

/* stream ids of the key material and of an encryption */
#define POLY_SECRET 1ull
#define POLY_PK_A 2ull
#define POLY_PK_E 3ull
#define POLY_KSK(kid, t) (0x1000000ull + (uint64_t)(kid) * 16ull + (uint64_t)(t))
#define POLY_ENC_V 0x2000001ull
#define POLY_ENC_E0 0x2000002ull
#define POLY_ENC_E1 0x2000003ull

/* ------------------------------------------------------------------------ */
/* objects                                                                    */
/* ------------------------------------------------------------------------ */
static or_ct *ct_alloc(const or_ctx *c, int level, double scale) {
    or_ct *x = malloc(sizeof *x);
    x->level = level;
    x->scale = scale;
    x->c = calloc((size_t)2 * (level + 1) * c->N, 8);
    return x;
}
static or_pt *pt_alloc(const or_ctx *c, int level, double scale) {
    or_pt *x = malloc(sizeof *x);
    x->level = level;
    x->scale = scale;
    x->m = calloc((size_t)(level + 1) * c->N, 8);
    return x;
}
#define CT0(c, x, i) ((x)->c + (size_t)(i) * (c)->N)
#define CT1(c, x, i) ((x)->c + (size_t)((x)->level + 1 + (i)) * (c)->N)

void or_ct_free(or_ct *x) { if (x) { free(x->c); free(x); } }
void or_pt_free(or_pt *x) { if (x) { free(x->m); free(x); } }

or_ct *or_ct_import(const or_ctx *c, const uint64_t *d, int level, double scale) {
    if (level < 0 || level > c->L) { set_err("or_ct_import: bad level"); return NULL; }
    or_ct *x = ct_alloc(c, level, scale);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i <= level; i++)
            for (int k = 0; k < c->N; k++) {
                size_t o = ((size_t)p * (level + 1) + i) * c->N + k;
                x->c[o] = d[o] % c->mod[i];
            }
    return x;
}
or_ct *or_ct_copy(const or_ctx *c, const or_ct *a) {
    or_ct *x = ct_alloc(c, a->level, a->scale);
    memcpy(x->c, a->c, (size_t)2 * (a->level + 1) * c->N * 8);
    return x;
}
or_pt *or_pt_import(const or_ctx *c, const uint64_t *m, int level, double scale) {
    if (level < 0 || level > c->L) { set_err("or_pt_import: bad level"); return NULL; }
    or_pt *x = pt_alloc(c, level, scale);
    for (int i = 0; i <= level; i++)
        for (int k = 0; k < c->N; k++) x->m[(size_t)i * c->N + k] = m[(size_t)i * c->N + k] % c->mod[i];
    return x;
}

/* ------------------------------------------------------------------------ */
/* keys (§3.2 encryption; §3.4.2 rotation = automorphism + key switch).      */
/* Reading: hybrid key switching with dnum digits of alpha consecutive       */
/* ciphertext primes and the CRT-idempotent gadget; digit t of the key for   */
/* s' is b_t = -a_t s + e_t + [P]_{q_i} s' on the limbs q_i of digit t, and   */
/* b_t = -a_t s + e_t on every other limb (P = 0 mod p_j).                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t kid;
    uint64_t *coef; /* [dnum][2][nmod][N] */
    uint64_t *ntt;  /* same, oracle NTT form, for the inner products */
} or_ksk;

struct or_keys {
    int64_t *s;       /* N ternary coefficients */
    uint64_t *s_res;  /* [nmod][N] */
    uint64_t *s_ntt;  /* [nmod][N] */
    uint64_t *pk;     /* [2][L+1][N] */
    int nksk;
    or_ksk *ksk;
};

const int64_t *or_keys_secret(const or_keys *k) { return k->s; }
const uint64_t *or_keys_pk(const or_keys *k) { return k->pk; }
static const or_ksk *find_ksk(const or_keys *k, uint64_t kid) {
    for (int i = 0; i < k->nksk; i++)
        if (k->ksk[i].kid == kid) return &k->ksk[i];
    return NULL;
}
const uint64_t *or_keys_ksk(const or_keys *k, uint64_t kid) {
    const or_ksk *x = find_ksk(k, kid);
    return x ? x->coef : NULL;
}

/* s_prime: [L+1][N] residues of the target key on the ciphertext primes */
static void make_ksk(const or_ctx *c, uint64_t seed, const or_keys *K, uint64_t kid,
                     const uint64_t *s_prime, or_ksk *out) {
    const int N = c->N, nm = c->nmod, L = c->L;
    out->kid = kid;
    out->coef = calloc((size_t)c->dnum * 2 * nm * N, 8);
    out->ntt = calloc((size_t)c->dnum * 2 * nm * N, 8);
    for (int t = 0; t < c->dnum; t++) {
        int64_t *e = malloc(8 * (size_t)N);
        or_sample_gauss(seed, POLY_KSK(kid, t), N, e);
        #pragma omp parallel for schedule(dynamic)
        for (int m = 0; m < nm; m++) {
            uint64_t q = c->mod[m];
            uint64_t *b = out->coef + (((size_t)t * 2 + 0) * nm + m) * N;
            uint64_t *a = out->coef + (((size_t)t * 2 + 1) * nm + m) * N;
            or_sample_uniform(seed, POLY_KSK(kid, t), m, q, N, a);
            uint64_t *as = malloc(8 * (size_t)N);
            or_polymul(c, m, a, K->s_res + (size_t)m * N, as);
            int in_digit = (m <= L) && (m >= t * c->alpha) && (m < (t + 1) * c->alpha);
            uint64_t Pmod = 1;
            if (in_digit)
                for (int j = 0; j < c->nP; j++) Pmod = mulmod(Pmod, c->mod[L + 1 + j] % q, q);
            for (int k = 0; k < N; k++) {
                uint64_t v = submod(smod(e[k], q), as[k], q);
                if (in_digit) v = addmod(v, mulmod(Pmod, s_prime[(size_t)m * N + k], q), q);
                b[k] = v;
            }
            free(as);
            uint64_t *bn = out->ntt + (((size_t)t * 2 + 0) * nm + m) * N;
            uint64_t *an = out->ntt + (((size_t)t * 2 + 1) * nm + m) * N;
            memcpy(bn, b, 8 * (size_t)N);
            memcpy(an, a, 8 * (size_t)N);
            nega_fwd(c, m, bn);
            nega_fwd(c, m, an);
        }
        free(e);
    }
}

or_keys *or_keygen(const or_ctx *c, uint64_t seed, const int32_t *rots, int nrot) {
    const int N = c->N, nm = c->nmod, L = c->L;
    or_keys *K = calloc(1, sizeof *K);
    K->s = malloc(8 * (size_t)N);
    or_sample_ternary(seed, POLY_SECRET, N, K->s);
    K->s_res = malloc(8 * (size_t)nm * N);
    K->s_ntt = malloc(8 * (size_t)nm * N);
    for (int m = 0; m < nm; m++)
        for (int k = 0; k < N; k++) K->s_res[(size_t)m * N + k] = smod(K->s[k], c->mod[m]);
    memcpy(K->s_ntt, K->s_res, 8 * (size_t)nm * N);
    for (int m = 0; m < nm; m++) nega_fwd(c, m, K->s_ntt + (size_t)m * N);
    /* public key (b, a) = (-a s + e, a) mod Q_L */
    K->pk = malloc(8 * (size_t)2 * (L + 1) * N);
    int64_t *e = malloc(8 * (size_t)N);
    or_sample_gauss(seed, POLY_PK_E, N, e);
    for (int m = 0; m <= L; m++) {
        uint64_t q = c->mod[m];
        uint64_t *b = K->pk + (size_t)m * N, *a = K->pk + (size_t)(L + 1 + m) * N;
        or_sample_uniform(seed, POLY_PK_A, m, q, N, a);
        uint64_t *as = malloc(8 * (size_t)N);
        or_polymul(c, m, a, K->s_res + (size_t)m * N, as);
        for (int k = 0; k < N; k++) b[k] = submod(smod(e[k], q), as[k], q);
        free(as);
    }
    free(e);
    /* distinct Galois elements of the requested rotations, plus s^2 (kid 0) */
    uint64_t *kids = malloc(sizeof(uint64_t) * (nrot + 1));
    int nk = 0;
    kids[nk++] = 0;
    for (int r = 0; r < nrot; r++) {
        uint64_t g = or_galois_element(c, rots[r]);
        if (g == 1) continue; /* rotation by 0 needs no key */
        int dup = 0;
        for (int i = 0; i < nk; i++) dup |= (kids[i] == g);
        if (!dup) kids[nk++] = g;
    }
    K->nksk = nk;
    K->ksk = calloc(nk, sizeof(or_ksk));
    uint64_t *sp = malloc(8 * (size_t)(L + 1) * N);
    for (int i = 0; i < nk; i++) {
        for (int m = 0; m <= L; m++) {
            uint64_t *dst = sp + (size_t)m * N;
            if (kids[i] == 0) or_polymul(c, m, K->s_res + (size_t)m * N, K->s_res + (size_t)m * N, dst);
            else or_automorphism(c, m, kids[i], K->s_res + (size_t)m * N, dst);
        }
        make_ksk(c, seed, K, kids[i], sp, &K->ksk[i]);
    }
    free(sp);
    free(kids);
    return K;
}

void or_keys_free(or_keys *K) {
    if (!K) return;
    for (int i = 0; i < K->nksk; i++) { free(K->ksk[i].coef); free(K->ksk[i].ntt); }
    free(K->ksk); free(K->s); free(K->s_res); free(K->s_ntt); free(K->pk); free(K);
}

/* ------------------------------------------------------------------------ */
/* encoding (§3.2): m_k = round(scale * (2/N) * sum_j z_j cos(pi e_jk / N)),  */
/* e_jk = 5^j k mod 2N -- the inverse of the canonical embedding             */
/* tau(m)_j = m(zeta^(5^j)), zeta = exp(i pi / N), for a real slot vector.    */
/* Rounding is to nearest, ties to even.                                     */
/* ------------------------------------------------------------------------ */
static int store_rounded(const or_ctx *c, const double *x, or_pt *p) {
    int N = c->N;
    for (int k = 0; k < N; k++) {
        double r = nearbyint(x[k]);
        if (!(fabs(r) < 9.2e18)) { set_err("or_encode: coefficient exceeds 2^63"); return -1; }
        int64_t v = (int64_t)r;
        for (int i = 0; i <= p->level; i++) p->m[(size_t)i * N + k] = smod(v, c->mod[i]);
    }
    return 0;
}

or_pt *or_encode_direct(const or_ctx *c, const double *z, int n, int level, double scale) {
    int N = c->N, h = N / 2;
    if (n > h || level < 0 || level > c->L) { set_err("or_encode: bad arguments"); return NULL; }
    double *x = malloc(sizeof(double) * N);
    #pragma omp parallel for
    for (int k = 0; k < N; k++) {
        double s = 0.0;
        for (int j = 0; j < n; j++) {
            uint64_t e = (c->pow5[j] * (uint64_t)k) % (2ull * N);
            s += z[j] * c->costab[e];
        }
        x[k] = scale * (2.0 / (double)N) * s;
    }
    or_pt *p = pt_alloc(c, level, scale);
    if (store_rounded(c, x, p)) { free(x); or_pt_free(p); return NULL; }
    free(x);
    return p;
}

/* Recursive radix-2 complex DFT: X[k] = sum_t x[t] exp(sign 2 pi i t k / n). */
static void fft_rec(double complex *x, int n, int sign, double complex *tmp) {
    if (n == 1) return;
    int h = n / 2;
    for (int i = 0; i < h; i++) { tmp[i] = x[2 * i]; tmp[h + i] = x[2 * i + 1]; }
    memcpy(x, tmp, sizeof(double complex) * n);
    fft_rec(x, h, sign, tmp);
    fft_rec(x + h, h, sign, tmp);
    for (int k = 0; k < h; k++) {
        double ang = sign * 2.0 * M_PI * (double)k / (double)n;
        double complex w = cos(ang) + I * sin(ang);
        double complex a = x[k], b = w * x[h + k];
        x[k] = a + b;
        x[h + k] = a - b;
    }
}

/* The same map through a length-N complex DFT.  The N roots zeta^(2t+1) carry
 * w[t]: slot j sits at 2t+1 = 5^j mod 2N and its conjugate at 2N - 5^j; then
 * m_k = Re(zeta^-k * DFT(w)[k]) / N. */
or_pt *or_encode_fft(const or_ctx *c, const double *z, int n, int level, double scale) {
    int N = c->N, h = N / 2;
    if (n > h || level < 0 || level > c->L) { set_err("or_encode: bad arguments"); return NULL; }
    double complex *w = calloc(N, sizeof(double complex)), *tmp = malloc(sizeof(double complex) * N);
    for (int j = 0; j < h; j++) {
        double v = j < n ? z[j] : 0.0;
        uint64_t e = c->pow5[j];
        w[(e - 1) / 2] = v;
        w[(2ull * N - e - 1) / 2] = v;
    }
    fft_rec(w, N, -1, tmp);
    double *x = malloc(sizeof(double) * N);
    for (int k = 0; k < N; k++) {
        double ang = -M_PI * (double)k / (double)N;
        double re = creal((cos(ang) + I * sin(ang)) * w[k]);
        x[k] = scale * re / (double)N;
    }
    free(w); free(tmp);
    or_pt *p = pt_alloc(c, level, scale);
    if (store_rounded(c, x, p)) { free(x); or_pt_free(p); return NULL; }
    free(x);
    return p;
}

or_pt *or_encode(const or_ctx *c, const double *z, int n, int level, double scale) {
    return c->logN <= 13 ? or_encode_direct(c, z, n, level, scale) : or_encode_fft(c, z, n, level, scale);
}

/* m = sum_i [m_i Qhat_i^-1]_{q_i} Qhat_i mod Q, centered into (-Q/2, Q/2]. */
int or_pt_lift(const or_ctx *c, const or_pt *p, double *out) {
    int l = p->level, N = c->N;
    big Q, halfQ, *Qhat = malloc(sizeof(big) * (l + 1));
    uint64_t *qhat_inv = malloc(8 * (size_t)(l + 1));
    big_zero(&Q); Q.w[0] = 1;
    for (int i = 0; i <= l; i++) big_mul_small(&Q, c->mod[i]);
    halfQ = Q;
    for (int i = 0; i < BW; i++) /* halfQ = floor(Q/2) */
        halfQ.w[i] = (halfQ.w[i] >> 1) | (i + 1 < BW ? (halfQ.w[i + 1] << 63) : 0);
    for (int i = 0; i <= l; i++) {
        big_zero(&Qhat[i]); Qhat[i].w[0] = 1;
        uint64_t prod = 1;
        for (int j = 0; j <= l; j++) {
            if (j == i) continue;
            big_mul_small(&Qhat[i], c->mod[j]);
            prod = mulmod(prod, c->mod[j] % c->mod[i], c->mod[i]);
        }
        qhat_inv[i] = invmod(prod, c->mod[i]);
    }
    #pragma omp parallel for
    for (int k = 0; k < N; k++) {
        big acc, t;
        big_zero(&acc);
        for (int i = 0; i <= l; i++) {
            uint64_t y = mulmod(p->m[(size_t)i * N + k], qhat_inv[i], c->mod[i]);
            t = Qhat[i];
            big_mul_small(&t, y);
            big_add(&acc, &t);
        }
        while (big_cmp(&acc, &Q) >= 0) big_sub(&acc, &Q);
        if (big_cmp(&acc, &halfQ) > 0) {
            t = Q;
            big_sub(&t, &acc);
            out[k] = -big_to_double(&t);
        } else {
            out[k] = big_to_double(&acc);
        }
    }
    free(Qhat); free(qhat_inv);
    return 0;
}

/* decode: z_j = Re m(zeta^(5^j)) / scale = sum_k m_k cos(pi e_jk / N) / scale */
int or_decode_direct(const or_ctx *c, const or_pt *p, double *z) {
    int N = c->N, h = N / 2;
    double *m = malloc(sizeof(double) * N);
    or_pt_lift(c, p, m);
    #pragma omp parallel for
    for (int j = 0; j < h; j++) {
        double s = 0.0;
        for (int k = 0; k < N; k++) {
            uint64_t e = (c->pow5[j] * (uint64_t)k) % (2ull * N);
            s += m[k] * c->costab[e];
        }
        z[j] = s / p->scale;
    }
    free(m);
    return 0;
}
/* the same through an inverse DFT: m(zeta^(2t+1)) = IDFT(m_k zeta^k)[t] * N */
int or_decode_fft(const or_ctx *c, const or_pt *p, double *z) {
    int N = c->N, h = N / 2;
    double *m = malloc(sizeof(double) * N);
    or_pt_lift(c, p, m);
    double complex *w = malloc(sizeof(double complex) * N), *tmp = malloc(sizeof(double complex) * N);
    for (int k = 0; k < N; k++) {
        double ang = M_PI * (double)k / (double)N;
        w[k] = m[k] * (cos(ang) + I * sin(ang));
    }
    fft_rec(w, N, +1, tmp);
    for (int j = 0; j < h; j++) z[j] = creal(w[(c->pow5[j] - 1) / 2]) / p->scale;
    free(m); free(w); free(tmp);
    return 0;
}
int or_decode(const or_ctx *c, const or_pt *p, double *z) {
    return c->logN <= 13 ? or_decode_direct(c, p, z) : or_decode_fft(c, p, z);
}

/* ------------------------------------------------------------------------ */
/* encrypt / decrypt (§3.2)                                                   */
/* ------------------------------------------------------------------------ */
/* ct = (v b + e0 + m, v a + e1) mod Q_l with pk = (b, a); v ternary,
 * e0, e1 Gaussian, all drawn from the encryption seed. */
or_ct *or_encrypt(const or_ctx *c, const or_keys *K, const or_pt *p, uint64_t seed) {
    int N = c->N, l = p->level, L = c->L;
    int64_t *v = malloc(8 * (size_t)N), *e0 = malloc(8 * (size_t)N), *e1 = malloc(8 * (size_t)N);
    or_sample_ternary(seed, POLY_ENC_V, N, v);
    or_sample_gauss(seed, POLY_ENC_E0, N, e0);
    or_sample_gauss(seed, POLY_ENC_E1, N, e1);
    or_ct *x = ct_alloc(c, l, p->scale);
    #pragma omp parallel for
    for (int i = 0; i <= l; i++) {
        uint64_t q = c->mod[i];
        uint64_t *vr = malloc(8 * (size_t)N), *t = malloc(8 * (size_t)N);
        for (int k = 0; k < N; k++) vr[k] = smod(v[k], q);
        or_polymul(c, i, vr, K->pk + (size_t)i * N, t);
        for (int k = 0; k < N; k++)
            CT0(c, x, i)[k] = addmod(addmod(t[k], smod(e0[k], q), q), p->m[(size_t)i * N + k], q);
        or_polymul(c, i, vr, K->pk + (size_t)(L + 1 + i) * N, t);
        for (int k = 0; k < N; k++) CT1(c, x, i)[k] = addmod(t[k], smod(e1[k], q), q);
        free(vr); free(t);
    }
    free(v); free(e0); free(e1);
    return x;
}

/* m = c0 + c1 s mod Q_l */
or_pt *or_decrypt(const or_ctx *c, const or_keys *K, const or_ct *x) {
    int N = c->N, l = x->level;
    or_pt *p = pt_alloc(c, l, x->scale);
    #pragma omp parallel for
    for (int i = 0; i <= l; i++) {
        uint64_t q = c->mod[i];
        uint64_t *t = malloc(8 * (size_t)N);
        or_polymul(c, i, CT1(c, x, i), K->s_res + (size_t)i * N, t);
        for (int k = 0; k < N; k++) p->m[(size_t)i * N + k] = addmod(CT0(c, x, i)[k], t[k], q);
        free(t);
    }
    return p;
}

/* ------------------------------------------------------------------------ */
/* basis conversion and key switching                                        */
/* ------------------------------------------------------------------------ */
/* global modulus index of position e of the extended basis Q_l U P */
static int ext_gidx(const or_ctx *c, int l, int e) { return e <= l ? e : c->L + 1 + (e - l - 1); }

/* Fast base conversion of digit t (ciphertext primes t*alpha ..
 * min(t*alpha+alpha, l+1)-1, product D) to every other modulus r of Q_l U P:
 *   y_r = sum_{i in digit} [x_i * (D/q_i)^-1]_{q_i} * (D/q_i mod r)  mod r,
 * with no overflow correction; on the digit's own limbs y = x.  Reading of
 * the digit decomposition of §3.4.2 as the RNS hybrid key switch. */
int or_modup_digit(const or_ctx *c, int l, int t, const uint64_t *x, uint64_t *out) {
    int N = c->N, nE = l + 1 + c->nP;
    int lo = t * c->alpha, hi = lo + c->alpha;
    if (hi > l + 1) hi = l + 1;
    if (lo >= hi) { set_err("or_modup_digit: empty digit"); return -1; }
    int nd = hi - lo;
    uint64_t dinv[64];
    for (int i = lo; i < hi; i++) {
        uint64_t prod = 1, qi = c->mod[i];
        for (int j = lo; j < hi; j++)
            if (j != i) prod = mulmod(prod, c->mod[j] % qi, qi);
        dinv[i - lo] = invmod(prod, qi);
    }
    #pragma omp parallel for
    for (int e = 0; e < nE; e++) {
        int g = ext_gidx(c, l, e);
        uint64_t *o = out + (size_t)e * N;
        if (g >= lo && g < hi) { memcpy(o, x + (size_t)g * N, 8 * (size_t)N); continue; }
        uint64_t r = c->mod[g];
        uint64_t dhat[64];
        for (int i = lo; i < hi; i++) {
            uint64_t prod = 1;
            for (int j = lo; j < hi; j++)
                if (j != i) prod = mulmod(prod, c->mod[j] % r, r);
            dhat[i - lo] = prod;
        }
        for (int k = 0; k < N; k++) {
            uint64_t acc = 0;
            for (int d = 0; d < nd; d++) {
                int i = lo + d;
                uint64_t y = mulmod(x[(size_t)i * N + k], dinv[d], c->mod[i]);
                acc = addmod(acc, mulmod(y, dhat[d], r), r);
            }
            o[k] = acc;
        }
    }
    return 0;
}

/* ModDown (rounded): out_i = (u - [u]_P^{+-}) * P^-1 mod q_i, where [u]_P^{+-}
 * is the centered residue of u modulo P in (-P/2, P/2]; i.e. out = round(u / P)
 * coefficient-wise, the same rounding rule as the rescale by one prime.
 * [u]_P is rebuilt exactly with big integers from the P limbs by the CRT:
 * X = sum_j [u_j (P/p_j)^-1]_{p_j} (P/p_j), reduced into [0, P), then centered.
 * Reading: the paper does not state the basis conversion; the uncentered
 * variant (floor(u/P) minus up to nP) leaves a one-sided bias per coefficient
 * that, multiplied by s, concentrates in the slots near the root 1. */
int or_moddown(const or_ctx *c, int l, const uint64_t *u, uint64_t *out) {
    int N = c->N, nP = c->nP, L = c->L;
    big P, halfP;
    big *Phat = malloc(sizeof(big) * nP);
    uint64_t phat_inv[64];
    big_zero(&P); P.w[0] = 1;
    for (int j = 0; j < nP; j++) big_mul_small(&P, c->mod[L + 1 + j]);
    halfP = P;
    for (int i = 0; i < BW; i++) halfP.w[i] = (halfP.w[i] >> 1) | (i + 1 < BW ? (halfP.w[i + 1] << 63) : 0);
    for (int j = 0; j < nP; j++) {
        uint64_t pj = c->mod[L + 1 + j], prod = 1;
        big_zero(&Phat[j]); Phat[j].w[0] = 1;
        for (int jj = 0; jj < nP; jj++) {
            if (jj == j) continue;
            big_mul_small(&Phat[j], c->mod[L + 1 + jj]);
            prod = mulmod(prod, c->mod[L + 1 + jj] % pj, pj);
        }
        phat_inv[j] = invmod(prod, pj);
    }
    uint64_t Pinv[64];
    for (int i = 0; i <= l; i++) {
        uint64_t q = c->mod[i], Pm = 1;
        for (int j = 0; j < nP; j++) Pm = mulmod(Pm, c->mod[L + 1 + j] % q, q);
        Pinv[i] = invmod(Pm, q);
    }
    #pragma omp parallel for
    for (int k = 0; k < N; k++) {
        big X, t;
        big_zero(&X);
        for (int j = 0; j < nP; j++) {
            uint64_t pj = c->mod[L + 1 + j];
            uint64_t y = mulmod(u[(size_t)(l + 1 + j) * N + k], phat_inv[j], pj);
            t = Phat[j];
            big_mul_small(&t, y);
            big_add(&X, &t);
        }
        while (big_cmp(&X, &P) >= 0) big_sub(&X, &P);
        int neg = big_cmp(&X, &halfP) > 0;  /* X > (P-1)/2: centered value X - P < 0 */
        if (neg) { t = P; big_sub(&t, &X); X = t; }  /* X = |centered value| */
        for (int i = 0; i <= l; i++) {
            uint64_t q = c->mod[i];
            uint64_t r = 0; /* |centered| mod q, Horner over the words */
            for (int w = BW - 1; w >= 0; w--) {
                u128 acc = ((u128)r << 64) | X.w[w];
                r = (uint64_t)(acc % q);
            }
            uint64_t vq = neg ? (r ? q - r : 0) : r;
            out[(size_t)i * N + k] = mulmod(submod(u[(size_t)i * N + k], vq, q), Pinv[i], q);
        }
    }
    free(Phat);
    return 0;
}

/* Accumulate sum_t sigma_g(ModUp_t(x)) * ksk_t into (U0, U1) over the
 * extended basis of level l (oracle NTT form).  g = 1 means no automorphism. */
static int ks_accumulate(const or_ctx *c, int l, const uint64_t *x, uint64_t g, const or_ksk *key,
                         uint64_t *U0, uint64_t *U1) {
    int N = c->N, nE = l + 1 + c->nP, nm = c->nmod;
    int ndig = (l + 1 + c->alpha - 1) / c->alpha;
    uint64_t *D = malloc(8 * (size_t)nE * N);
    for (int t = 0; t < ndig; t++) {
        if (or_modup_digit(c, l, t, x, D)) { free(D); return -1; }
        #pragma omp parallel for
        for (int e = 0; e < nE; e++) {
            int gm = ext_gidx(c, l, e);
            uint64_t q = c->mod[gm];
            uint64_t *tmp = malloc(8 * (size_t)N);
            if (g != 1) or_automorphism(c, gm, g, D + (size_t)e * N, tmp);
            else memcpy(tmp, D + (size_t)e * N, 8 * (size_t)N);
            nega_fwd(c, gm, tmp);
            const uint64_t *kb = key->ntt + (((size_t)t * 2 + 0) * nm + gm) * N;
            const uint64_t *ka = key->ntt + (((size_t)t * 2 + 1) * nm + gm) * N;
            uint64_t *u0 = U0 + (size_t)e * N, *u1 = U1 + (size_t)e * N;
            for (int k = 0; k < N; k++) {
                u0[k] = addmod(u0[k], mulmod(tmp[k], kb[k], q), q);
                u1[k] = addmod(u1[k], mulmod(tmp[k], ka[k], q), q);
            }
            free(tmp);
        }
    }
    free(D);
    return 0;
}
/* back from the oracle NTT form and ModDown to Q_l; adds into (o0, o1) */
static void ks_finish(const or_ctx *c, int l, uint64_t *U0, uint64_t *U1, uint64_t *o0, uint64_t *o1) {
    int N = c->N, nE = l + 1 + c->nP;
    #pragma omp parallel for
    for (int e = 0; e < nE; e++) {
        int gm = ext_gidx(c, l, e);
        nega_inv(c, gm, U0 + (size_t)e * N);
        nega_inv(c, gm, U1 + (size_t)e * N);
    }
    uint64_t *d0 = malloc(8 * (size_t)(l + 1) * N), *d1 = malloc(8 * (size_t)(l + 1) * N);
    or_moddown(c, l, U0, d0);
    or_moddown(c, l, U1, d1);
    for (int i = 0; i <= l; i++) {
        uint64_t q = c->mod[i];
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            o0[o] = addmod(o0[o], d0[o], q);
            o1[o] = addmod(o1[o], d1[o], q);
        }
    }
    free(d0); free(d1);
}

/* Hoisted rotations (§3.4.2): for each k, with g = 5^k mod 2N,
 *   Rot_k(ct) = (sigma_g(c0) + ModDown(U0), ModDown(U1)),
 *   U = sum_t sigma_g(ModUp_t(c1)) * ksk_{g,t}.
 * The automorphism is applied after ModUp, to the extended digits. */
int or_rotate_hoisted(const or_ctx *c, const or_keys *K, const or_ct *x, const int32_t *rots,
                      int nrot, or_ct **out) {
    int N = c->N, l = x->level, nE = l + 1 + c->nP;
    for (int r = 0; r < nrot; r++) {
        uint64_t g = or_galois_element(c, rots[r]);
        if (g != 1 && !find_ksk(K, g)) { set_err("or_rotate_hoisted: missing rotation key"); return -1; }
    }
    for (int r = 0; r < nrot; r++) {
        uint64_t g = or_galois_element(c, rots[r]);
        or_ct *y = ct_alloc(c, l, x->scale);
        if (g == 1) {
            memcpy(y->c, x->c, (size_t)2 * (l + 1) * N * 8);
            out[r] = y;
            continue;
        }
        for (int i = 0; i <= l; i++) or_automorphism(c, i, g, CT0(c, x, i), CT0(c, y, i));
        uint64_t *U0 = calloc((size_t)nE * N, 8), *U1 = calloc((size_t)nE * N, 8);
        ks_accumulate(c, l, CT1(c, x, 0), g, find_ksk(K, g), U0, U1);
        ks_finish(c, l, U0, U1, CT0(c, y, 0), CT1(c, y, 0));
        free(U0); free(U1);
        out[r] = y;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* rescale, arithmetic                                                        */
/* ------------------------------------------------------------------------ */
/* Rescale (§3.2, multiplication paragraph): drop q_l,
 *   c'_i = (c_i - [c_l]^{+-}) * q_l^-1 mod q_i,  [.]^{+-} centered in (-q_l/2, q_l/2];
 * this equals round(c / q_l) coefficient-wise.  scale /= q_l. */
or_ct *or_rescale(const or_ctx *c, const or_ct *a) {
    int N = c->N, l = a->level;
    if (l < 1) { set_err("or_rescale: level 0"); return NULL; }
    uint64_t ql = c->mod[l];
    or_ct *y = ct_alloc(c, l - 1, a->scale / (double)ql);
    for (int p = 0; p < 2; p++) {
        const uint64_t *top = (p ? CT1(c, a, l) : CT0(c, a, l));
        for (int i = 0; i < l; i++) {
            uint64_t q = c->mod[i], qinv = invmod(ql % q, q);
            const uint64_t *src = p ? CT1(c, a, i) : CT0(c, a, i);
            uint64_t *dst = p ? CT1(c, y, i) : CT0(c, y, i);
            for (int k = 0; k < N; k++) {
                uint64_t x = top[k];
                int64_t centered = (x > ql / 2) ? -(int64_t)(ql - x) : (int64_t)x;
                dst[k] = mulmod(submod(src[k], smod(centered, q), q), qinv, q);
            }
        }
    }
    return y;
}

static int same_shape(const or_ct *a, const or_ct *b) { return a->level == b->level; }

or_ct *or_add(const or_ctx *c, const or_ct *a, const or_ct *b) {
    if (!same_shape(a, b)) { set_err("or_add: level mismatch"); return NULL; }
    or_ct *y = ct_alloc(c, a->level, a->scale);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i <= a->level; i++) {
            const uint64_t *x0 = p ? CT1(c, a, i) : CT0(c, a, i), *x1 = p ? CT1(c, b, i) : CT0(c, b, i);
            uint64_t *d = p ? CT1(c, y, i) : CT0(c, y, i);
            for (int k = 0; k < c->N; k++) d[k] = addmod(x0[k], x1[k], c->mod[i]);
        }
    return y;
}
or_ct *or_sub(const or_ctx *c, const or_ct *a, const or_ct *b) {
    if (!same_shape(a, b)) { set_err("or_sub: level mismatch"); return NULL; }
    or_ct *y = ct_alloc(c, a->level, a->scale);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i <= a->level; i++) {
            const uint64_t *x0 = p ? CT1(c, a, i) : CT0(c, a, i), *x1 = p ? CT1(c, b, i) : CT0(c, b, i);
            uint64_t *d = p ? CT1(c, y, i) : CT0(c, y, i);
            for (int k = 0; k < c->N; k++) d[k] = submod(x0[k], x1[k], c->mod[i]);
        }
    return y;
}
/* plaintext x ciphertext product (§3.2): both components times m */
or_ct *or_mul_plain(const or_ctx *c, const or_ct *a, const or_pt *p) {
    int l = a->level < p->level ? a->level : p->level;
    or_ct *y = ct_alloc(c, l, a->scale * p->scale);
    #pragma omp parallel for
    for (int i = 0; i <= l; i++) {
        or_polymul(c, i, CT0(c, a, i), p->m + (size_t)i * c->N, CT0(c, y, i));
        or_polymul(c, i, CT1(c, a, i), p->m + (size_t)i * c->N, CT1(c, y, i));
    }
    return y;
}
or_ct *or_mul_int(const or_ctx *c, const or_ct *a, int64_t kc) {
    or_ct *y = ct_alloc(c, a->level, a->scale * (double)kc);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i <= a->level; i++) {
            uint64_t q = c->mod[i], kq = smod(kc, q);
            const uint64_t *x = p ? CT1(c, a, i) : CT0(c, a, i);
            uint64_t *d = p ? CT1(c, y, i) : CT0(c, y, i);
            for (int k = 0; k < c->N; k++) d[k] = mulmod(x[k], kq, q);
        }
    return y;
}
or_ct *or_add_const(const or_ctx *c, const or_ct *a, double cst) {
    or_ct *y = or_ct_copy(c, a);
    int64_t v = (int64_t)nearbyint(cst * a->scale);
    for (int i = 0; i <= a->level; i++) {
        uint64_t q = c->mod[i];
        CT0(c, y, i)[0] = addmod(CT0(c, y, i)[0], smod(v, q), q);
    }
    return y;
}
or_ct *or_drop_to(const or_ctx *c, const or_ct *a, int level) {
    if (level > a->level || level < 0) { set_err("or_drop_to: bad level"); return NULL; }
    or_ct *y = ct_alloc(c, level, a->scale);
    for (int i = 0; i <= level; i++) {
        memcpy(CT0(c, y, i), CT0(c, a, i), 8 * (size_t)c->N);
        memcpy(CT1(c, y, i), CT1(c, a, i), 8 * (size_t)c->N);
    }
    return y;
}

/* ct x ct (§3.2 multiplication): tensor (a0b0, a0b1 + a1b0, a1b1), then
 * relinearise d2 with the key for s^2, then rescale.  Scale a.s * b.s / q_l. */
/* Encrypted-database product (§3.3.1 encrypts the diagonal rows; §3.4.1's
 * deferred relinearisation): the tensor products (a0 b0, a0 b1 + a1 b0,
 * a1 b1) of n ciphertext pairs are summed as a degree-2 ciphertext, which is
 * relinearised once with the s^2 key and rescaled. */
or_ct *or_tensor_sum_relin_rescale(const or_ctx *c, const or_keys *K, const or_ct *const *a, const or_ct *const *b,
                                   int n) {
    if (n < 1) { set_err("or_tensor_sum: no pairs"); return NULL; }
    for (int t = 0; t < n; t++)
        if (!same_shape(a[t], a[0]) || !same_shape(b[t], a[0])) { set_err("or_tensor_sum: level mismatch"); return NULL; }
    const or_ksk *rk = find_ksk(K, 0);
    if (!rk) { set_err("or_tensor_sum: missing relinearisation key"); return NULL; }
    int N = c->N, l = a[0]->level, nE = l + 1 + c->nP;
    or_ct *y = ct_alloc(c, l, a[0]->scale * b[0]->scale);
    uint64_t *d2 = calloc((size_t)(l + 1) * N, 8);
    #pragma omp parallel for
    for (int i = 0; i <= l; i++) {
        uint64_t q = c->mod[i];
        uint64_t *t = malloc(8 * (size_t)N);
        uint64_t *y0 = CT0(c, y, i), *y1 = CT1(c, y, i), *z2 = d2 + (size_t)i * N;
        for (int k = 0; k < N; k++) y0[k] = y1[k] = 0;
        for (int p = 0; p < n; p++) {
            or_polymul(c, i, CT0(c, a[p], i), CT0(c, b[p], i), t);
            for (int k = 0; k < N; k++) y0[k] = addmod(y0[k], t[k], q);
            or_polymul(c, i, CT0(c, a[p], i), CT1(c, b[p], i), t);
            for (int k = 0; k < N; k++) y1[k] = addmod(y1[k], t[k], q);
            or_polymul(c, i, CT1(c, a[p], i), CT0(c, b[p], i), t);
            for (int k = 0; k < N; k++) y1[k] = addmod(y1[k], t[k], q);
            or_polymul(c, i, CT1(c, a[p], i), CT1(c, b[p], i), t);
            for (int k = 0; k < N; k++) z2[k] = addmod(z2[k], t[k], q);
        }
        free(t);
    }
    uint64_t *U0 = calloc((size_t)nE * N, 8), *U1 = calloc((size_t)nE * N, 8);
    ks_accumulate(c, l, d2, 1, rk, U0, U1);
    ks_finish(c, l, U0, U1, CT0(c, y, 0), CT1(c, y, 0));
    free(U0); free(U1); free(d2);
    or_ct *z = or_rescale(c, y);
    or_ct_free(y);
    return z;
}

or_ct *or_mul_relin_rescale(const or_ctx *c, const or_keys *K, const or_ct *a, const or_ct *b) {
    if (!same_shape(a, b)) { set_err("or_mul_relin: level mismatch"); return NULL; }
    const or_ksk *rk = find_ksk(K, 0);
    if (!rk) { set_err("or_mul_relin: missing relinearisation key"); return NULL; }
    int N = c->N, l = a->level, nE = l + 1 + c->nP;
    or_ct *y = ct_alloc(c, l, a->scale * b->scale);
    uint64_t *d2 = malloc(8 * (size_t)(l + 1) * N);
    #pragma omp parallel for
    for (int i = 0; i <= l; i++) {
        uint64_t q = c->mod[i];
        uint64_t *t0 = malloc(8 * (size_t)N), *t1 = malloc(8 * (size_t)N);
        or_polymul(c, i, CT0(c, a, i), CT0(c, b, i), CT0(c, y, i));
        or_polymul(c, i, CT0(c, a, i), CT1(c, b, i), t0);
        or_polymul(c, i, CT1(c, a, i), CT0(c, b, i), t1);
        for (int k = 0; k < N; k++) CT1(c, y, i)[k] = addmod(t0[k], t1[k], q);
        or_polymul(c, i, CT1(c, a, i), CT1(c, b, i), d2 + (size_t)i * N);
        free(t0); free(t1);
    }
    uint64_t *U0 = calloc((size_t)nE * N, 8), *U1 = calloc((size_t)nE * N, 8);
    ks_accumulate(c, l, d2, 1, rk, U0, U1);
    ks_finish(c, l, U0, U1, CT0(c, y, 0), CT1(c, y, 0));
    free(U0); free(U1); free(d2);
    or_ct *z = or_rescale(c, y);
    or_ct_free(y);
    return z;
}

/* ------------------------------------------------------------------------ */
/* database of pre-rotated diagonals (§3.3.1 packing, Eq. diag, Eq.          */
/* prerotation of §5.3.1 applied to the plaintext slot vector as in §5.3.3)   */
/* ------------------------------------------------------------------------ */
struct or_db {
    int N, G, ell, B, n1, level;
    double scale;
    or_pt **pt;       /* [G*ell] */
    uint64_t **ntt;   /* [G*ell] oracle NTT form, [level+1][N] */
    uint64_t **ntt_p; /* [G*ell] residues mod the special primes, oracle NTT form, [nP][N]; built on first use */
};

int or_db_groups(const or_db *db) { return db->G; }

/* Slot vector of diagonal d of group g before encoding.  Block b of the
 * group holds templates (g B + b) ell + r, row r at slot b ell + r;
 * diag_d[b ell + r] = T[(g B + b) ell + r][(r + d) mod ell]; slots past
 * B ell are zero; then the whole N/2-slot vector is rotated by -j n1
 * (d = j n1 + i): v[s] = diag_d[(s - j n1) mod N/2]. */
int or_db_slots(const or_ctx *c, const float *T, int K, int ell, int B, int n1, int g, int d, double *v) {
    int h = c->N / 2;
    if (ell <= 0 || B <= 0 || (long)B * ell > h || d < 0 || d >= ell || n1 <= 0) {
        set_err("or_db_slots: bad layout");
        return -1;
    }
    int j = d / n1;
    for (int s = 0; s < h; s++) {
        int src = ((s - j * n1) % h + h) % h;
        double val = 0.0;
        if (src < B * ell) {
            int b = src / ell, r = src % ell;
            long row = ((long)g * B + b) * ell + r;
            if (row < K) val = (double)T[row * ell + (r + d) % ell];
        }
        v[s] = val;
    }
    return 0;
}

static void db_cache_ntt(const or_ctx *c, or_db *db) {
    int N = c->N, n = db->G * db->ell;
    db->ntt = calloc(n, sizeof(uint64_t *));
    #pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < n; p++) {
        db->ntt[p] = malloc(8 * (size_t)(db->level + 1) * N);
        memcpy(db->ntt[p], db->pt[p]->m, 8 * (size_t)(db->level + 1) * N);
        for (int i = 0; i <= db->level; i++) nega_fwd(c, i, db->ntt[p] + (size_t)i * N);
    }
}

or_db *or_db_build(const or_ctx *c, const float *T, int K, int ell, int B, int n1, int level, double scale_d) {
    int h = c->N / 2;
    if (K < 0 || ell <= 0 || B <= 0 || (long)B * ell > h || n1 <= 0 || n1 > ell || level < 0 || level > c->L) {
        set_err("or_db_build: bad arguments");
        return NULL;
    }
    or_db *db = calloc(1, sizeof *db);
    db->N = c->N;
    db->ell = ell; db->B = B; db->n1 = n1; db->level = level; db->scale = scale_d;
    db->G = (K + B * ell - 1) / (B * ell);
    if (db->G < 1) db->G = 1;
    int n = db->G * ell, fail = 0;
    db->pt = calloc(n, sizeof(or_pt *));
    #pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < n; p++) {
        double *v = malloc(sizeof(double) * h);
        or_db_slots(c, T, K, ell, B, n1, p / ell, p % ell, v);
        db->pt[p] = or_encode(c, v, h, level, scale_d);
        if (!db->pt[p]) fail = 1;
        free(v);
    }
    if (fail) { or_db_free(db); return NULL; }
    db_cache_ntt(c, db);
    return db;
}

or_db *or_db_import(const or_ctx *c, const uint64_t *coeffs, int G, int ell, int B, int n1, int level, double scale_d) {
    if (G < 1 || ell <= 0 || n1 <= 0 || n1 > ell || level < 0 || level > c->L) {
        set_err("or_db_import: bad arguments");
        return NULL;
    }
    or_db *db = calloc(1, sizeof *db);
    db->N = c->N;
    db->G = G; db->ell = ell; db->B = B; db->n1 = n1; db->level = level; db->scale = scale_d;
    db->pt = calloc((size_t)G * ell, sizeof(or_pt *));
    size_t per = (size_t)(level + 1) * c->N;
    for (int p = 0; p < G * ell; p++) db->pt[p] = or_pt_import(c, coeffs + per * p, level, scale_d);
    db_cache_ntt(c, db);
    return db;
}

void or_db_free(or_db *db) {
    if (!db) return;
    int n = db->G * db->ell;
    for (int p = 0; p < n; p++) {
        if (db->pt) or_pt_free(db->pt[p]);
        if (db->ntt) free(db->ntt[p]);
        if (db->ntt_p) free(db->ntt_p[p]);
    }
    free(db->pt); free(db->ntt); free(db->ntt_p); free(db);
}

/* The plaintext's integer coefficients modulo the special primes p_j: each
 * coefficient m is rebuilt exactly from its Q_level limbs by the CRT,
 * m = sum_i [m_i Qhat_i^-1]_{q_i} Qhat_i mod Q, taken as the centered value in
 * (-Q/2, Q/2], and reduced mod p_j (coefficient form, [nP][N]).  A plaintext
 * multiplied into a ciphertext held over Q_l U P needs these limbs. */
static void pt_special_residues(const or_ctx *c, const or_pt *p, uint64_t *out) {
    int l = p->level, N = c->N, nP = c->nP, L = c->L;
    big Q, halfQ, *Qhat = malloc(sizeof(big) * (l + 1));
    uint64_t *qhat_inv = malloc(8 * (size_t)(l + 1));
    big_zero(&Q); Q.w[0] = 1;
    for (int i = 0; i <= l; i++) big_mul_small(&Q, c->mod[i]);
    halfQ = Q;
    for (int i = 0; i < BW; i++) halfQ.w[i] = (halfQ.w[i] >> 1) | (i + 1 < BW ? (halfQ.w[i + 1] << 63) : 0);
    for (int i = 0; i <= l; i++) {
        big_zero(&Qhat[i]); Qhat[i].w[0] = 1;
        uint64_t prod = 1;
        for (int j = 0; j <= l; j++) {
            if (j == i) continue;
            big_mul_small(&Qhat[i], c->mod[j]);
            prod = mulmod(prod, c->mod[j] % c->mod[i], c->mod[i]);
        }
        qhat_inv[i] = invmod(prod, c->mod[i]);
    }
    #pragma omp parallel for
    for (int k = 0; k < N; k++) {
        big X, t;
        big_zero(&X);
        for (int i = 0; i <= l; i++) {
            t = Qhat[i];
            big_mul_small(&t, mulmod(p->m[(size_t)i * N + k], qhat_inv[i], c->mod[i]));
            big_add(&X, &t);
        }
        while (big_cmp(&X, &Q) >= 0) big_sub(&X, &Q);
        int neg = big_cmp(&X, &halfQ) > 0;
        if (neg) { t = Q; big_sub(&t, &X); X = t; }  /* X = |m| */
        for (int j = 0; j < nP; j++) {
            uint64_t pj = c->mod[L + 1 + j], r = 0;
            for (int w = BW - 1; w >= 0; w--) r = (uint64_t)((((u128)r << 64) | X.w[w]) % pj);
            out[(size_t)j * N + k] = neg ? (r ? pj - r : 0) : r;
        }
    }
    free(Qhat); free(qhat_inv);
}

static void db_cache_ntt_p(const or_ctx *c, or_db *db) {
    if (db->ntt_p) return;
    int N = c->N, n = db->G * db->ell, nP = c->nP, L = c->L;
    db->ntt_p = calloc(n, sizeof(uint64_t *));
    for (int p = 0; p < n; p++) {
        db->ntt_p[p] = malloc(8 * (size_t)nP * N);
        pt_special_residues(c, db->pt[p], db->ntt_p[p]);
        for (int j = 0; j < nP; j++) nega_fwd(c, L + 1 + j, db->ntt_p[p] + (size_t)j * N);
    }
}

/* Builds the special-prime limbs of every diagonal now (else on first use). */
int or_db_extend(const or_ctx *c, or_db *db) {
    db_cache_ntt_p(c, db);
    return 0;
}

int or_db_export_special(const or_ctx *c, or_db *db, int g, int d, uint64_t *out) {
    if (g < 0 || g >= db->G || d < 0 || d >= db->ell) { set_err("or_db_export_special: bad index"); return -1; }
    pt_special_residues(c, db->pt[(size_t)g * db->ell + d], out);
    return 0;
}

int or_db_export(const or_db *db, int g, int d, uint64_t *out) {
    if (g < 0 || g >= db->G || d < 0 || d >= db->ell) { set_err("or_db_export: bad index"); return -1; }
    const or_pt *p = db->pt[(size_t)g * db->ell + d];
    memcpy(out, p->m, 8 * (size_t)(p->level + 1) * (size_t)db->N);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* BSGS matrix-vector product with pre-rotated diagonals (Eq. bsgs2, §3.4;   */
/* Eq. prerotation, §5.3.1; Alg. gpu-bsgs-index, §5.4).                       */
/*   P_j = sum_{i < min(n1, ell - j n1)} baby[i] * diag'_{g, j n1 + i}        */
/*   P_j <- Rescale(P_j)                    (rescale before the giant step)   */
/*   S_g = P_0 + sum_{j >= 1} Rot_{j n1}(P_j)                                 */
/* The giant rotations share one ModDown: U = sum_j sum_t sigma_{g_j}(       */
/* ModUp_t(P_j.c1)) * ksk_{g_j,t};  S = (P_0.c0 + sum_j sigma_{g_j}(P_j.c0)   */
/* + ModDown(U0), P_0.c1 + ModDown(U1)).                                      */
/* ------------------------------------------------------------------------ */
static or_ct *giant_sum(const or_ctx *c, const or_keys *K, or_ct **P, int n2, int n1);

or_ct *or_bsgs_matvec(const or_ctx *c, const or_keys *K, or_ct *const *baby, int n1, const or_db *db, int group) {
    int N = c->N, ell = db->ell;
    if (n1 != db->n1 || group < 0 || group >= db->G) { set_err("or_bsgs_matvec: layout mismatch"); return NULL; }
    int lv = baby[0]->level;
    for (int i = 0; i < n1; i++)
        if (baby[i]->level != lv || baby[i]->scale != baby[0]->scale) {
            set_err("or_bsgs_matvec: baby steps differ in level or scale");
            return NULL;
        }
    if (db->level < lv) lv = db->level;
    if (lv < 1) { set_err("or_bsgs_matvec: no level left to rescale"); return NULL; }
    int n2 = (ell + n1 - 1) / n1;
    for (int j = 1; j < n2; j++)
        if (!find_ksk(K, or_galois_element(c, j * n1))) { set_err("or_bsgs_matvec: missing giant-step key"); return NULL; }
    /* baby steps in oracle NTT form, restricted to level lv */
    uint64_t **bn = malloc(sizeof(uint64_t *) * n1);
    for (int i = 0; i < n1; i++) {
        bn[i] = malloc(8 * (size_t)2 * (lv + 1) * N);
        for (int p = 0; p < 2; p++)
            for (int m = 0; m <= lv; m++) {
                uint64_t *d = bn[i] + ((size_t)p * (lv + 1) + m) * N;
                memcpy(d, p ? CT1(c, baby[i], m) : CT0(c, baby[i], m), 8 * (size_t)N);
                nega_fwd(c, m, d);
            }
    }
    or_ct **P = calloc(n2, sizeof(or_ct *));
    for (int j = 0; j < n2; j++) {
        int nb = ell - j * n1 < n1 ? ell - j * n1 : n1;
        or_ct *acc = ct_alloc(c, lv, baby[0]->scale * db->scale);
        #pragma omp parallel for
        for (int pm = 0; pm < 2 * (lv + 1); pm++) {
            int p = pm / (lv + 1), m = pm % (lv + 1);
            uint64_t q = c->mod[m];
            uint64_t *d = p ? CT1(c, acc, m) : CT0(c, acc, m);
            for (int i = 0; i < nb; i++) {
                const uint64_t *x = bn[i] + ((size_t)p * (lv + 1) + m) * N;
                const uint64_t *w = db->ntt[(size_t)group * ell + j * n1 + i] + (size_t)m * N;
                for (int k = 0; k < N; k++) d[k] = addmod(d[k], mulmod(x[k], w[k], q), q);
            }
            nega_inv(c, m, d);
        }
        P[j] = or_rescale(c, acc);
        or_ct_free(acc);
    }
    for (int i = 0; i < n1; i++) free(bn[i]);
    free(bn);
    return giant_sum(c, K, P, n2, n1);
}

/* S = P_0 + sum_{j >= 1} Rot_{j n1}(P_j) with one shared ModDown (the giant
 * steps of Eq. bsgs2); frees P. */
static or_ct *giant_sum(const or_ctx *c, const or_keys *K, or_ct **P, int n2, int n1) {
    int N = c->N, l = P[0]->level, nE = l + 1 + c->nP;
    or_ct *S = or_ct_copy(c, P[0]);
    uint64_t *U0 = calloc((size_t)nE * N, 8), *U1 = calloc((size_t)nE * N, 8);
    uint64_t *tmp = malloc(8 * (size_t)N);
    for (int j = 1; j < n2; j++) {
        uint64_t g = or_galois_element(c, j * n1);
        for (int i = 0; i <= l; i++) {
            or_automorphism(c, i, g, CT0(c, P[j], i), tmp);
            for (int k = 0; k < N; k++) CT0(c, S, i)[k] = addmod(CT0(c, S, i)[k], tmp[k], c->mod[i]);
        }
        ks_accumulate(c, l, CT1(c, P[j], 0), g, find_ksk(K, g), U0, U1);
    }
    if (n2 > 1) ks_finish(c, l, U0, U1, CT0(c, S, 0), CT1(c, S, 0));
    free(tmp); free(U0); free(U1);
    for (int j = 0; j < n2; j++) or_ct_free(P[j]);
    free(P);
    return S;
}

/* S = P[0] + sum_{j >= 1} Rot_{j stride}(P[j]) for n ciphertexts of one
 * level and scale: the giant-step rotate-sum of Eq. bsgs2 (§3.4) on its own,
 * as the on-demand giant rotations of §5.3.2 apply it to the inner sums of
 * an encrypted database.  The inputs are left as they are. */
or_ct *or_rotate_sum(const or_ctx *c, const or_keys *K, const or_ct *const *P, int n, int stride) {
    if (n < 1) { set_err("or_rotate_sum: no input"); return NULL; }
    for (int j = 0; j < n; j++)
        if (!same_shape(P[j], P[0]) || P[j]->scale != P[0]->scale) { set_err("or_rotate_sum: inputs differ"); return NULL; }
    for (int j = 1; j < n; j++)
        if (!find_ksk(K, or_galois_element(c, j * stride))) { set_err("or_rotate_sum: missing rotation key"); return NULL; }
    or_ct **Q = malloc(sizeof(or_ct *) * (size_t)n);
    for (int j = 0; j < n; j++) Q[j] = or_ct_copy(c, P[j]);
    return giant_sum(c, K, Q, n, stride);
}

/* BSGS product with the ModDown of the baby steps hoisted past the inner
 * sums, and that of the inner sums' first polynomials past the giant-step
 * sum (double hoisting of the plaintext-matrix BSGS, §3.4.2 hoisting and
 * double hoisting).  Baby step i is kept over the extended basis Q_l U P,
 *   B_i = (P sigma_i(c0) + U0_i, U1_i),  U_i = sum_t sigma_i(ModUp_t(c1)) ksk_{i,t},
 *   B_0 = (P c0, P c1)  (zero on the special primes),
 * the diagonals are multiplied over Q_l U P (their special-prime limbs are
 * the residues of the plaintext's centered integer coefficients) into the
 * inner sums A_j = sum_i B_i * diag'_{g, j n1 + i} = (a_j, b_j).  A rotation
 * acts on a_j without a key, so the first polynomials are rotated and summed
 * over Q_l U P and take one ModDown and one rescale together; each b_j takes
 * its own, and the giant steps key-switch them:
 *   S = (Rescale(ModDown(sum_j sigma_{j n1}(a_j))), Rescale(ModDown(b_0)))
 *       + sum_{j >= 1} KeySwitch_{j n1}(sigma_{j n1}(Rescale(ModDown(b_j)))),
 * the key switches sharing one ModDown as in or_bsgs_matvec.  ModDown(B_i) is
 * Rot_i(ct), so the result approximates the same product. */
or_ct *or_bsgs_matvec_hoisted(const or_ctx *c, const or_keys *K, const or_ct *x, int n1, or_db *db, int group) {
    int N = c->N, ell = db->ell, l = x->level, nP = c->nP;
    if (n1 != db->n1 || group < 0 || group >= db->G) { set_err("or_bsgs_matvec_hoisted: layout mismatch"); return NULL; }
    if (db->level != l) { set_err("or_bsgs_matvec_hoisted: query and database levels differ"); return NULL; }
    if (l < 1) { set_err("or_bsgs_matvec_hoisted: no level left to rescale"); return NULL; }
    int n2 = (ell + n1 - 1) / n1, nE = l + 1 + nP;
    for (int i = 1; i < n1; i++)
        if (!find_ksk(K, or_galois_element(c, i))) { set_err("or_bsgs_matvec_hoisted: missing baby-step key"); return NULL; }
    for (int j = 1; j < n2; j++)
        if (!find_ksk(K, or_galois_element(c, j * n1))) { set_err("or_bsgs_matvec_hoisted: missing giant-step key"); return NULL; }
    db_cache_ntt_p(c, db);
    uint64_t Pq[64];
    for (int i = 0; i <= l; i++) {
        Pq[i] = 1;
        for (int j = 0; j < nP; j++) Pq[i] = mulmod(Pq[i], c->mod[c->L + 1 + j] % c->mod[i], c->mod[i]);
    }
    /* baby steps over Q_l U P, oracle NTT form, [2][nE][N] each */
    uint64_t **bq = malloc(sizeof(uint64_t *) * n1);
    for (int i = 0; i < n1; i++) {
        uint64_t g = or_galois_element(c, i);
        uint64_t *b0 = calloc((size_t)2 * nE * N, 8), *b1 = b0 + (size_t)nE * N;
        bq[i] = b0;
        if (g != 1) ks_accumulate(c, l, CT1(c, x, 0), g, find_ksk(K, g), b0, b1);
        #pragma omp parallel for
        for (int e = 0; e <= l; e++) {
            uint64_t q = c->mod[e], *t = malloc(8 * (size_t)N);
            if (g != 1) or_automorphism(c, e, g, CT0(c, x, e), t);
            else memcpy(t, CT0(c, x, e), 8 * (size_t)N);
            nega_fwd(c, e, t);
            for (int k = 0; k < N; k++) b0[(size_t)e * N + k] = addmod(b0[(size_t)e * N + k], mulmod(Pq[e], t[k], q), q);
            if (g == 1) {
                memcpy(t, CT1(c, x, e), 8 * (size_t)N);
                nega_fwd(c, e, t);
                for (int k = 0; k < N; k++) b1[(size_t)e * N + k] = mulmod(Pq[e], t[k], q);
            }
            free(t);
        }
    }
    or_ct **P = calloc(n2, sizeof(or_ct *));
    uint64_t *acc = malloc(8 * (size_t)2 * nE * N);
    uint64_t *asum = calloc((size_t)nE * N, 8), *b0 = malloc(8 * (size_t)nE * N);
    double scale = x->scale * db->scale;
    for (int j = 0; j < n2; j++) {
        int nb = ell - j * n1 < n1 ? ell - j * n1 : n1;
        memset(acc, 0, 8 * (size_t)2 * nE * N);
        #pragma omp parallel for
        for (int pe = 0; pe < 2 * nE; pe++) {
            int e = pe % nE, gm = ext_gidx(c, l, e);
            uint64_t q = c->mod[gm], *d = acc + (size_t)pe * N;
            for (int i = 0; i < nb; i++) {
                size_t di = (size_t)group * ell + j * n1 + i;
                const uint64_t *w = e <= l ? db->ntt[di] + (size_t)e * N : db->ntt_p[di] + (size_t)(e - l - 1) * N;
                const uint64_t *xb = bq[i] + (size_t)pe * N;
                for (int k = 0; k < N; k++) d[k] = addmod(d[k], mulmod(xb[k], w[k], q), q);
            }
            nega_inv(c, gm, d);
        }
        /* a_j: rotated by j n1 and summed over Q_l U P (coefficient form) */
        uint64_t g = or_galois_element(c, j * n1);
        #pragma omp parallel for
        for (int e = 0; e < nE; e++) {
            int gm = ext_gidx(c, l, e);
            uint64_t q = c->mod[gm], *t = malloc(8 * (size_t)N);
            or_automorphism(c, gm, g, acc + (size_t)e * N, t);
            for (int k = 0; k < N; k++) asum[(size_t)e * N + k] = addmod(asum[(size_t)e * N + k], t[k], q);
            free(t);
        }
        /* b_j: its own ModDown and rescale (b_0 joins the final ciphertext) */
        if (j == 0) {
            memcpy(b0, acc + (size_t)nE * N, 8 * (size_t)nE * N);
        } else {
            or_ct *y = ct_alloc(c, l, scale);
            or_moddown(c, l, acc + (size_t)nE * N, CT1(c, y, 0));
            P[j] = or_rescale(c, y);  /* (0, Rescale(ModDown(b_j))) */
            or_ct_free(y);
        }
    }
    or_ct *y = ct_alloc(c, l, scale);
    or_moddown(c, l, asum, CT0(c, y, 0));
    or_moddown(c, l, b0, CT1(c, y, 0));
    P[0] = or_rescale(c, y);
    or_ct_free(y);
    free(acc); free(asum); free(b0);
    for (int i = 0; i < n1; i++) free(bq[i]);
    free(bq);
    /* the giant steps of or_bsgs_matvec: the first polynomials of P[j >= 1]
     * are zero, so only the key switches of the b_j add to P[0] */
    return giant_sum(c, K, P, n2, n1);
}

/* ------------------------------------------------------------------------ */
/* Chebyshev threshold (§5.1.4, Eq. cheb-sign)                                */
/* ------------------------------------------------------------------------ */
/* Interpolant of f(x) = 1 if x >= delta else 0 at the n+1 first-kind nodes
 * x_j = cos(pi (j + 1/2) / (n+1)) ("DCT-based interpolation"):
 *   c_k = (2/(n+1)) sum_j f(x_j) cos(pi k (j + 1/2) / (n+1)),  c_0 halved,
 * so that p = sum_k c[k] T_k. */
void or_cheb_step_coeffs(int n, double delta, double *c) {
    int m = n + 1;
    for (int k = 0; k <= n; k++) {
        double s = 0.0;
        for (int j = 0; j < m; j++) {
            double xj = cos(M_PI * ((double)j + 0.5) / (double)m);
            double f = xj >= delta ? 1.0 : 0.0;
            s += f * cos(M_PI * (double)k * ((double)j + 0.5) / (double)m);
        }
        c[k] = 2.0 * s / (double)m;
    }
    c[0] *= 0.5;
}

/* Clenshaw's recurrence for sum_k c[k] T_k(x). */
double or_cheb_clenshaw(const double *c, int n, double x) {
    double b1 = 0.0, b2 = 0.0;
    for (int k = n; k >= 1; k--) {
        double b0 = 2.0 * x * b1 - b2 + c[k];
        b2 = b1;
        b1 = b0;
    }
    return x * b1 - b2 + c[0];
}

/* Homomorphic evaluation.  The paper evaluates the series with
 * Paterson-Stockmeyer over baby-step powers T_1..T_{d1} and giant powers
 * T_{d1 2^j} (§5.1.4); its printed algorithm does not hold in the Chebyshev
 * basis as written, so the reading taken is the Chebyshev-basis division
 *   p = q T_M + r,  q_0 = c_M, q_i = 2 c_{M+i},  r_0 = c_0,
 *   r_k = c_k - c_{2M-k},  M = d1 2^j the largest with M < (#coefficients),
 * recursing on q and r down to leaves of fewer than d1 + 1 coefficients.
 * Every power comes from T_i = 2 T_ceil(i/2) T_floor(i/2) - T_(i mod 2).
 *
 * Scale rule: every ciphertext at level l carries the canonical scale
 * D[l], D[l0] = input scale, D[l-1] = D[l]^2 / q_l.  A real constant c
 * multiplies a level-l ciphertext as the integer round(c D[l-1] q_l / D[l])
 * followed by a rescale; a level change from l to lam < l drops to lam+1
 * and multiplies by round(D[lam] q_{lam+1} / D[l]) before rescaling. */
typedef struct {
    const or_ctx *c;
    const or_keys *K;
    double D[OR_MAXMOD];
    int d1;
    or_ct **T;
    int nT;
    int nmul;
    int fail;
} cheb_state;

static int64_t rne_i64(double x) { return (int64_t)nearbyint(x); }

/* bring a to level lam with the canonical scale (consumes one extra level) */
static or_ct *cheb_adjust(cheb_state *st, const or_ct *a, int lam) {
    const or_ctx *c = st->c;
    if (a->level == lam) return or_ct_copy(c, a);
    if (lam < 0 || lam > a->level) { st->fail = 1; set_err("or_chebyshev: not enough levels"); return NULL; }
    or_ct *d = or_drop_to(c, a, lam + 1);
    int64_t k = rne_i64((st->D[lam] * (double)c->mod[lam + 1]) / st->D[a->level]);
    or_ct *m = or_mul_int(c, d, k);
    or_ct *r = or_rescale(c, m);
    r->scale = st->D[lam];
    or_ct_free(d); or_ct_free(m);
    return r;
}
static or_ct *cheb_mul(cheb_state *st, const or_ct *a, const or_ct *b) {
    int lam = a->level < b->level ? a->level : b->level;
    if (lam < 1) { st->fail = 1; set_err("or_chebyshev: not enough levels"); return NULL; }
    or_ct *x = cheb_adjust(st, a, lam), *y = cheb_adjust(st, b, lam);
    or_ct *z = (x && y) ? or_mul_relin_rescale(st->c, st->K, x, y) : NULL;
    if (!z) { st->fail = 1; or_ct_free(x); or_ct_free(y); return NULL; }
    z->scale = st->D[lam - 1];
    st->nmul++;
    or_ct_free(x); or_ct_free(y);
    return z;
}
static or_ct *cheb_add_matched(cheb_state *st, const or_ct *a, const or_ct *b) {
    int lam = a->level < b->level ? a->level : b->level;
    or_ct *x = cheb_adjust(st, a, lam), *y = cheb_adjust(st, b, lam);
    or_ct *z = (x && y) ? or_add(st->c, x, y) : NULL;
    or_ct_free(x); or_ct_free(y);
    return z;
}
static const or_ct *cheb_power(cheb_state *st, int i) {
    if (st->T[i]) return st->T[i];
    int a = (i + 1) / 2, b = i / 2;
    const or_ct *Ta = cheb_power(st, a);
    const or_ct *Tb = cheb_power(st, b);
    if (st->fail) return NULL;
    or_ct *prod = cheb_mul(st, Ta, Tb);
    if (!prod) return NULL;
    or_ct *two = or_add(st->c, prod, prod);
    or_ct *res;
    if (a == b) {
        res = or_add_const(st->c, two, -1.0);
    } else {
        or_ct *t1 = cheb_adjust(st, st->T[1], two->level);
        res = t1 ? or_sub(st->c, two, t1) : NULL;
        or_ct_free(t1);
    }
    or_ct_free(prod); or_ct_free(two);
    st->T[i] = res;
    return res;
}
/* c times T (one level) */
static or_ct *cheb_scalar(cheb_state *st, const or_ct *T, double cst) {
    const or_ctx *c = st->c;
    int lv = T->level, lam = lv - 1;
    if (lam < 0) { st->fail = 1; set_err("or_chebyshev: not enough levels"); return NULL; }
    int64_t k = rne_i64(((cst * st->D[lam]) * (double)c->mod[lv]) / st->D[lv]);
    or_ct *m = or_mul_int(c, T, k);
    or_ct *r = or_rescale(c, m);
    r->scale = st->D[lam];
    or_ct_free(m);
    return r;
}
/* sum_{i<m} c[i] T_i for 2 <= m <= d1: one rescale for the whole sum */
static or_ct *cheb_leaf(cheb_state *st, const double *cf, int m) {
    const or_ctx *c = st->c;
    int lam = 1 << 30;
    for (int i = 1; i < m; i++) {
        const or_ct *Ti = cheb_power(st, i);
        if (!Ti) return NULL;
        if (Ti->level - 1 < lam) lam = Ti->level - 1;
    }
    if (lam < 0) { st->fail = 1; set_err("or_chebyshev: not enough levels"); return NULL; }
    or_ct *acc = NULL;
    for (int i = 1; i < m; i++) {
        or_ct *d = or_drop_to(c, st->T[i], lam + 1);
        int64_t k = rne_i64(((cf[i] * st->D[lam]) * (double)c->mod[lam + 1]) / st->D[st->T[i]->level]);
        or_ct *t = or_mul_int(c, d, k);
        or_ct_free(d);
        if (!acc) acc = t;
        else { or_ct *s = or_add(c, acc, t); or_ct_free(acc); or_ct_free(t); acc = s; }
    }
    or_ct *r = or_rescale(c, acc);
    r->scale = st->D[lam];
    or_ct_free(acc);
    or_ct *out = or_add_const(c, r, cf[0]);
    or_ct_free(r);
    return out;
}
static or_ct *cheb_eval(cheb_state *st, const double *cf, int m) {
    if (st->fail) return NULL;
    if (m <= st->d1) return cheb_leaf(st, cf, m);
    int M = st->d1;
    while (2 * M < m) M *= 2;
    int nq = m - M;
    double *q = malloc(sizeof(double) * nq), *r = malloc(sizeof(double) * M);
    q[0] = cf[M];
    for (int i = 1; i < nq; i++) q[i] = 2.0 * cf[M + i];
    r[0] = cf[0];
    for (int k = 1; k < M; k++) r[k] = cf[k] - ((2 * M - k < m) ? cf[2 * M - k] : 0.0);
    const or_ct *TM = cheb_power(st, M);
    or_ct *A = NULL;
    if (TM) {
        if (nq == 1) {
            A = cheb_scalar(st, TM, q[0]);
        } else {
            or_ct *Q = cheb_eval(st, q, nq);
            if (Q) { A = cheb_mul(st, Q, TM); or_ct_free(Q); }
        }
    }
    or_ct *R = A ? cheb_eval(st, r, M) : NULL;
    free(q); free(r);
    if (!A || !R) { st->fail = 1; or_ct_free(A); or_ct_free(R); return NULL; }
    or_ct *S = cheb_add_matched(st, A, R);
    or_ct_free(A); or_ct_free(R);
    return S;
}

or_ct *or_chebyshev(const or_ctx *c, const or_keys *K, const or_ct *x, const double *cf, int n, int d1) {
    if (n < 1 || d1 < 2) { set_err("or_chebyshev: need degree >= 1 and d1 >= 2"); return NULL; }
    cheb_state st;
    memset(&st, 0, sizeof st);
    st.c = c; st.K = K; st.d1 = d1;
    st.D[x->level] = x->scale;
    for (int l = x->level; l >= 1; l--) st.D[l - 1] = (st.D[l] * st.D[l]) / (double)c->mod[l];
    st.nT = n + 2 > 2 * d1 + 2 ? n + 2 : 2 * d1 + 2;
    st.T = calloc(st.nT, sizeof(or_ct *));
    st.T[1] = or_ct_copy(c, x);
    g_err[0] = 0;
    or_ct *y = cheb_eval(&st, cf, n + 1);
    for (int i = 0; i < st.nT; i++) or_ct_free(st.T[i]);
    free(st.T);
    if (!y && !g_err[0]) set_err("or_chebyshev: not enough levels");
    return y;
}

/* number of relinearised products of the recursion above (no ciphertexts) */
static int count_eval(int m, int d1, int *have, int *nm);
static void count_power(int i, int *have, int *nm) {
    if (have[i]) return;
    count_power((i + 1) / 2, have, nm);
    count_power(i / 2, have, nm);
    have[i] = 1;
    (*nm)++;
}
static int count_eval(int m, int d1, int *have, int *nm) {
    if (m <= d1) {
        for (int i = 1; i < m; i++) count_power(i, have, nm);
        return 0;
    }
    int M = d1;
    while (2 * M < m) M *= 2;
    count_power(M, have, nm);
    if (m - M > 1) { count_eval(m - M, d1, have, nm); (*nm)++; }
    count_eval(M, d1, have, nm);
    return 0;
}
int or_chebyshev_count_mults(int n, int d1) {
    int sz = n + 2 > 2 * d1 + 2 ? n + 2 : 2 * d1 + 2;
    int *have = calloc(sz, sizeof(int));
    have[1] = 1;
    int nm = 0;
    count_eval(n + 1, d1, have, &nm);
    free(have);
    return nm;
}

/* ------------------------------------------------------------------------ */
/* threads (for timing the oracle at a stated core count)                     */
/* ------------------------------------------------------------------------ */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }
