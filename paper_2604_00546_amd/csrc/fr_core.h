// fr_core.h -- internal declarations of the gfx950 library behind include/fr.h.
//
// Storage conventions (private to the library):
//  * every polynomial limb is N uint64 words holding a residue mod its prime,
//    canonical in [0, q), in the evaluation (NTT) domain in bit-reversed
//    order: word p of limb q_i is the value at psi_i^(2 brv(p) + 1);
//  * ciphertexts are [2][level+1][N] (c0 limbs, then c1 limbs);
//  * key-switching keys and database diagonals -- the constant operands of the
//    two multiply-accumulate kernels -- are stored pre-multiplied by 2^64 mod q
//    ("Montgomery-scaled"), so that a lazily accumulated 128-bit sum of
//    products reduces to the canonical result with one Montgomery reduction.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fr.h"

typedef uint64_t u64;
typedef uint32_t u32;

#define FR_MAXMOD 64
#define FR_MAXLEVEL 48
// multiword tables of the special modulus (at most 8 special primes below 2^60)
constexpr int kPbigWords = 9, kPbigRows = 9;

// ---------------------------------------------------------------------------
// per-modulus constants
// ---------------------------------------------------------------------------
struct ModConst {
    u64 q;
    u64 mu;        // floor(2^64 / q): Barrett quotient for 64-bit inputs
    u64 qinv_neg;  // -q^-1 mod 2^64: Montgomery
    u64 r64;       // 2^64 mod q
    u64 r64_sh;    // Shoup companion of r64
    u64 r128;      // 2^128 mod q
    u64 ninv;      // N^-1 mod q
    u64 ninv_sh;
};

// ---------------------------------------------------------------------------
// device modular arithmetic
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 mulhi64(u64 a, u64 b) { return __umul64hi(a, b); }

// x mod q for any 64-bit x (q < 2^62): quotient estimate is at most 1 short
__device__ __forceinline__ u64 reduce64(u64 x, const ModConst &m) {
    u64 r = x - mulhi64(x, m.mu) * m.q;
    return r >= m.q ? r - m.q : r;
}
// a * w mod q with the Shoup companion wp = floor(w 2^64 / q); any 64-bit a
__device__ __forceinline__ u64 shoup(u64 a, u64 w, u64 wp, u64 q) {
    u64 r = a * w - mulhi64(a, wp) * q;
    return r >= q ? r - q : r;
}
__device__ __forceinline__ u64 addq(u64 a, u64 b, u64 q) {
    u64 s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 subq(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// Montgomery reduction of (hi:lo) with hi < q: returns (hi:lo) 2^-64 mod q
__device__ __forceinline__ u64 redc(u64 lo, u64 hi, const ModConst &m) {
    u64 t = lo * m.qinv_neg;
    u64 r = hi + mulhi64(t, m.q) + (lo != 0 ? 1u : 0u);
    return r >= m.q ? r - m.q : r;
}
// 128-bit accumulator (hi:lo) of products with one Montgomery-scaled factor:
// returns (hi:lo) 2^-64 mod q for any hi
__device__ __forceinline__ u64 redc_any(u64 lo, u64 hi, const ModConst &m) {
    return redc(lo, reduce64(hi, m), m);
}
// canonical a * b mod q (a, b < q)
__device__ __forceinline__ u64 mulmod(u64 a, u64 b, const ModConst &m) {
    u64 lo = a * b, hi = mulhi64(a, b);
    return shoup(redc(lo, hi, m), m.r64, m.r64_sh, m.q);
}
// any 128-bit value mod q
__device__ __forceinline__ u64 reduce128(u64 lo, u64 hi, const ModConst &m) {
    return shoup(redc_any(lo, hi, m), m.r64, m.r64_sh, m.q);
}
// (hi:lo) += a * b
__device__ __forceinline__ void mac128(u64 &lo, u64 &hi, u64 a, u64 b) {
    u64 pl = a * b, ph = mulhi64(a, b);
    lo += pl;
    hi += ph + (lo < pl ? 1u : 0u);
}

__device__ __forceinline__ u32 brv(u32 x, int logN) { return __brev(x) >> (32 - logN); }
// evaluation-domain automorphism sigma_g: output word p reads input word
// brv(((2 brv(p) + 1) g mod 2N - 1) / 2)
__device__ __forceinline__ u32 auto_src(u32 p, u64 g, int logN) {
    u64 e = ((2ull * brv(p, logN) + 1ull) * g) & ((2ull << logN) - 1ull);
    return brv((u32)((e - 1) >> 1), logN);
}

// ---------------------------------------------------------------------------
// limb addressing inside a launch: launch limb y -> storage limb s ->
// global modulus index (Q limbs first, then P limbs)
// ---------------------------------------------------------------------------
struct LimbMap {
    int first;    // storage limb of launch limb 0
    int skip_lo;  // storage limbs [skip_lo, skip_lo + skip_n) are skipped
    int skip_n;
    int nq;       // storage limbs below nq are q_s; the rest are p_(s - nq)
    int pbase;    // global index of p_0 (= L + 1)
    __host__ __device__ int storage(int y) const {
        int s = first + y;
        return s >= skip_lo ? s + skip_n : s;
    }
    __host__ __device__ int modidx(int s) const { return s < nq ? s : pbase + (s - nq); }
};

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Arena {  // bump allocator over device chunks, reset per top-level call
    struct Chunk { char *base; size_t size, used; };
    std::vector<Chunk> chunks;
    size_t peak = 0;
    size_t limit = ~(size_t)0;  // most bytes the chunks may total
    int hold = 0;  // > 0: scopes do not give space back (work on several streams)
    void *get(size_t bytes);  // 256-byte aligned; nullptr on failure or past the limit
    size_t allocated() const;
    bool grow(size_t bytes);  // one more chunk of exactly `bytes` (within the limit)
    void reset();
    void release();
};
// thrown by the scratch allocator when the arena cannot grow; every entry
// point catches it and returns FR_ENOMEM
struct ArenaFull {
    size_t bytes, allocated, limit;
};
// restores the context's stream on scope exit (work spread over the
// auxiliary streams switches it temporarily)
struct StreamRestore {
    hipStream_t &slot;
    hipStream_t saved;
    explicit StreamRestore(hipStream_t &s) : slot(s), saved(s) {}
    ~StreamRestore() { slot = saved; }
};

// kernel timing hook: events around every launch of one kernel class
enum KernelClass { K_NONE = 0, K_NTT = 1, K_MODUP = 2, K_KS = 3, K_MODDOWN = 4, K_MAC = 5, K_RESCALE = 6,
                   K_TENSOR = 7, K_ELEM = 8 };
// Key-switching key storage: per (digit, b or a) a block of nmod limbs; the
// limb of a modulus below 2^40 holds 5 bytes per word (N low words, then N
// high bytes), the others 8.  The layout depends only on the moduli.
struct KeyLayout {
    unsigned off[FR_MAXMOD];
    unsigned char packed[FR_MAXMOD];
    size_t block;  // bytes per (digit, b or a) block
};

struct Prof {
    int cls = K_NONE;
    std::vector<hipEvent_t> ev;  // pairs
    int used = 0;
    double bytes = 0.0;
    bool begin(int k, hipStream_t s);
    void end(int k, hipStream_t s, double b);
};

struct fr_ctx {
    int logN, N, L, nP, dnum, alpha, nmod;
    u64 mod[FR_MAXMOD];
    ModConst hmod[FR_MAXMOD];
    ModConst *d_mod = nullptr;
    // twiddles [nmod][N]: psi^brv(k), Shoup companions, inverses
    u64 *d_tw = nullptr, *d_tw_sh = nullptr, *d_itw = nullptr, *d_itw_sh = nullptr;
    u64 *d_tw2 = nullptr, *d_itw2 = nullptr;  // interleaved (twiddle, companion) pairs [nmod][N][2]
    // ModUp tables, per (level, digit): dinv[nd], dinv_sh[nd], dhat[nE][nd]
    // (dhat Montgomery-scaled by 2^64 mod r_e)
    u64 *d_modup = nullptr;
    size_t modup_off[FR_MAXLEVEL][8];
    // ModDown tables: phat_inv[nP], phat_inv_sh[nP], phat_mod[L+1][nP]
    // (Montgomery-scaled by 2^64 mod q_i),
    // Pinv[L+1], Pinv_sh[L+1], P mod q_i [L+1], 1/p_j [nP] (double bits),
    // -e P 2^64 mod q_i [L+1][nP+1] (e = 0..nP), P 2^64 mod q_i [L+1]
    u64 *d_moddown = nullptr;
    // ModDown's exact overflow decision: [kPbigRows][kPbigWords] words, row
    // j < nP = Phat_j = P / p_j, row kPbigRows - 1 = P, little-endian 64-bit
    // words (zero-padded)
    u64 *d_pbig = nullptr;
    u64 P_mod_q[FR_MAXMOD], P_mod_q_sh[FR_MAXMOD];
    u64 P_inv_q[FR_MAXMOD], P_inv_q_sh[FR_MAXMOD];  // P^-1 mod q_i and Shoup companions
    // rescale: qinv[l][i] = q_l^-1 mod q_i and Shoup, [L+1][L+1] each; then
    // (P q_l)^-1 mod q_i in the same layout (ModDown and rescale in one product)
    u64 *d_rescale = nullptr;
    // CRT lift per level: qhat_inv[i], qhat_inv_sh[i], qhat_mod64[i], Q_mod64,
    // inv_q (double) -- laid out as [L+1][4 * (L+1) + 1] words
    u64 *d_crt = nullptr;
    // FFT twiddles exp(-2 pi i k / N), k < N/2, and zeta^k, k < N
    double *d_fft_w = nullptr, *d_zeta = nullptr;
    u32 *d_slot_pos = nullptr;  // (5^j mod 2N - 1) / 2, j < N/2
    u64 cdt[20];
    hipStream_t stream = nullptr;
    // auxiliary streams (default priority) and events for independent work
    // of one call that runs concurrently; joined into `stream` before return
    static const int kAux = 3;
    hipStream_t aux[kAux] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kAux] = {};
    // events marking finished groups of a recorded DAG: kDagEv / (1 + kAux)
    // slots per stream, taken in turn by the groups that stream runs, so a
    // slot is only ever re-recorded on the stream that recorded it before,
    // after the work it marked: a waiter that reads the newer record waits at
    // least as long as it needs to
    static const int kDagEv = 64;
    hipEvent_t ev_dag[kDagEv] = {};
    static_assert(kDagEv % (1 + kAux) == 0, "DAG event slots must split evenly over the streams");
    Arena arena;
    // fr_rotate_hoisted_noalloc: this device's fixed scratch array (its
    // address from hipGetSymbolAddress) as a one-chunk arena that never grows
    Arena fixed_arena;
    KeyLayout klay{};
    int *d_flag = nullptr;  // device error flag
    Prof *prof = nullptr;
    // tuning knobs (fr_ctx_set_tune; defaults are measured choices)
    int tune[FR_TUNE_COUNT] = {32, 32, 48, 48, 12, 8, 8, 1, 1, 1};
    // graph capture (fr_graph_begin / fr_graph_end): the calls of a capture
    // run on cap_stream in capture mode; arena_gen counts releases of the
    // arena, which invalidate graphs recorded before them
    hipStream_t cap_stream = nullptr, saved_stream = nullptr;
    bool capturing = false;
    unsigned arena_gen = 0;
};

// bracket a launch of class K with timing events when that class is selected
struct ProfScope {
    const fr_ctx *c;
    int k;
    double bytes;
    bool on;
    ProfScope(const fr_ctx *cc, int kk, double b) : c(cc), k(kk), bytes(b) {
        on = c->prof && c->prof->begin(k, c->stream);
    }
    ~ProfScope() {
        if (on) c->prof->end(k, c->stream, bytes);
    }
};

struct KeyEntry {
    u64 kid;
    unsigned char *data;  // [dnum][2] blocks of KeyLayout, eval domain, Montgomery-scaled
};

struct fr_keys {
    fr_ctx *ctx;
    u64 *s_eval = nullptr;   // [nmod][N] canonical eval-domain s
    u64 *s_mont = nullptr;   // [nmod][N] Montgomery-scaled s
    u64 *pk = nullptr;       // [2][L+1][N] eval domain canonical
    std::vector<KeyEntry> ksk;
    const KeyEntry *find(u64 kid) const {
        for (auto &k : ksk)
            if (k.kid == kid) return &k;
        return nullptr;
    }
};

// Byte layout of one diagonal: limb m at off[m]; a limb whose modulus is
// below 2^40 is packed (packed[m] = 1) as N low 32-bit words followed by N
// high bytes, any other as N 64-bit words.
constexpr int kDbMaxLimbs = 32;
struct DbLayout {
    unsigned off[kDbMaxLimbs];
    unsigned char packed[kDbMaxLimbs];
};

struct fr_db {
    fr_ctx *ctx;
    int G, ell, B, n1, level;
    int nl;  // limbs per diagonal: level+1, or level+1+nP once extended
    double scale;
    // [G][ell] diagonals of `stride` bytes each (layout `lay`), eval domain,
    // Montgomery-scaled; limbs 0..level are the q_i, the extended form
    // appends the special primes p_0..p_{nP-1}
    size_t stride = 0;
    DbLayout lay{};
    unsigned char *data = nullptr;
};

// ---------------------------------------------------------------------------
// host parameter math (params.cpp)
// ---------------------------------------------------------------------------
namespace frh {
u64 mulmod_h(u64 a, u64 b, u64 q);
u64 powmod_h(u64 b, u64 e, u64 q);
u64 invmod_h(u64 a, u64 q);
u64 shoup_companion(u64 w, u64 q);
bool is_prime(u64 n);
int choose_primes(int logN, int q0_bits, int n_mid, int mid_bits, int n_special, int special_bits,
                  u64 *out);
u64 primitive_2n_root(u64 q, int N);
ModConst make_modconst(u64 q, int N);
void gauss_cdt(u64 cdt[20]);
u64 galois_element(int N, int rot);
int ext_limbs(const fr_ctx *c, int level);    // level+1+nP
int num_digits(const fr_ctx *c, int level);   // ceil((level+1)/alpha)
}  // namespace frh

// ---------------------------------------------------------------------------
// kernel launchers (kernels_*.hip)
// ---------------------------------------------------------------------------
// one item of a batched integer linear combination: sources (ciphertexts
// [2][lp1][N]) with their signed integer factors
struct ScalarItem {
    std::vector<const u64 *> src;
    std::vector<long long> k;
    std::vector<int> lp1;
};

namespace frk {
// NTT over `nlimbs` limbs x `npoly` polynomials; poly_stride in words.  With
// src set the transform is out of place: it reads src (same limb map,
// src_poly_stride between polynomials) and writes data.
void ntt_fwd(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly, size_t poly_stride,
             const u64 *src = nullptr, size_t src_poly_stride = 0, int own_alpha = 0, int own_ndig = 1,
             int own_nlq = 0);
// whether ntt_fwd honours own_alpha (ModUp digit sets: polynomial z is digit
// z % own_ndig, whose own limbs are already in evaluation form and are left
// untouched); on other rings it transforms every limb
bool ntt_own_skip_ok(const fr_ctx *c);
// rescale fused into one forward transform (radix-16 kernels; returns false
// when the ring has no such kernels): out[p] = (in[p] - NTT(centered(xtop[p])
// mod q_i)) q_l^-1 for limbs i < l; xtop[p] is the coefficient form of limb l
// of polynomial p (N words each), tmp holds npoly * l limbs between passes
bool ntt_fwd_rescale(const fr_ctx *c, u64 *tmp, int l, int npoly, const u64 *xtop, const u64 *in, size_t in_stride,
                     u64 *out, size_t out_stride);
// ModDown finish fused into the forward transform of V (the converted
// correction, coefficient form, npoly polynomials of level+1 limbs):
// out[p] (+)= (U[p] - NTT(V[p])) P^-1 on limbs 0..level; U and out strides
// su / so per polynomial.  Returns false when the ring has no radix-16
// kernels.
bool ntt_fwd_moddown(const fr_ctx *c, u64 *V, int level, int npoly, const u64 *U, size_t su, u64 *out, size_t so,
                     bool accumulate);
// last step of a relinearised product merged with its rescale: out[p] =
// (d[p] + (U[p] - NTT(Z[p])) P^-1) q_l^-1 on limbs 0..l-1 (Z from
// relin_rescale_prep; d null: no d term, Rescale(ModDown(U))); false when
// the ring has no radix-16 kernels
bool ntt_fwd_relin_rescale(const fr_ctx *c, u64 *Z, int l, int npoly, const u64 *U, size_t su, const u64 *d,
                           size_t sd, u64 *out, size_t so);
void ntt_inv(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly, size_t poly_stride,
             const u64 *src = nullptr, size_t src_poly_stride = 0);

void add(const fr_ctx *c, u64 *out, const u64 *a, const u64 *b, int nlimbs, int npoly,
         size_t so, size_t sa, size_t sb, bool subtract);
// out[p][i] = a[p][i] * k_i (per-limb constants, Shoup)
void mul_const(const fr_ctx *c, u64 *out, const u64 *a, const u64 *k, const u64 *k_sh, int nlimbs,
               int npoly, size_t so, size_t sa);
// out[i] = a[i] + k_i on every word (constant polynomial in eval domain)
void add_const(const fr_ctx *c, u64 *out, const u64 *a, const u64 *k, int nlimbs);
// out[p][i] = a[p][i] * b[i] (b canonical, eval domain)
void mul_pt(const fr_ctx *c, u64 *out, const u64 *a, const u64 *b, int nlimbs, int npoly, size_t so,
            size_t sa);
// tensor: d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1
void tensor(const fr_ctx *c, u64 *d0, u64 *d1, u64 *d2, const u64 *a0, const u64 *a1, const u64 *b0,
            const u64 *b1, int nlimbs);
// out[i][p] = (accumulate ? out : 0) + in[i][auto_src(p, g)]
void automorph(const fr_ctx *c, u64 *out, const u64 *in, u64 g, int nlimbs, int npoly, size_t so,
               size_t si, bool accumulate);
// multiply every limb by 2^64 mod q (to Montgomery-scaled) or by 2^-64 (back)
void mont_scale(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly,
                size_t poly_stride, bool to_mont);
// fast base conversion of every digit of `batch` items at once: D[b][t] =
// [ndig][nE][N] per item (item stride sd).  The digit's own limbs are
// copied from own (the evaluation-form input, items so words apart) when
// given, else in coefficient form (a forward transform over all nE limbs
// then completes every digit)
void modup_all(const fr_ctx *c, u64 *D, const u64 *x, int level, int batch, size_t sd, size_t sx,
               const u64 *own = nullptr, size_t so = 0);
// fast base conversion of one digit: coefficient-form x[level+1][N] ->
// D[nE][N] coefficient form on every extended limb outside the digit; with
// own, the digit's own limbs of D are copied from own (items so words apart)
void modup_digit(const fr_ctx *c, u64 *D, const u64 *x, int level, int t, int batch = 1, size_t sd = 0,
                 size_t sx = 0, const u64 *own = nullptr, size_t so = 0);
// U{0,1}[e][p] (+)= sum_t D_t[e][auto_src(p, g)] * ksk_t{b,a}[gm(e)][p];
// with fold_d (relinearisation, items fold_sd words apart) the top limb e =
// level is replaced by d_l + P^-1 U_l (its only later use); with rot_c0
// (items c0_sd words apart, level+1 limbs) U0 also takes P c0[e][auto_src(p,
// g)] on the limbs e <= level: the rotation of (c0, c1) held over Q_l U P,
// before its ModDown
void ks_inner(const fr_ctx *c, u64 *U0, u64 *U1, const u64 *D, const unsigned char *ksk, u64 g, int level,
              bool accumulate, int batch = 1, size_t sd = 0, size_t su = 0, const u64 *fold_d = nullptr,
              size_t fold_sd = 0, const u64 *rot_c0 = nullptr, size_t c0_sd = 0);
// Baby steps of the hoisted product, nrot rotations at once: rotation r's
// outputs at U + r ub, (U0 over nE limbs, then U1), with P sigma_g(c0) folded
// into U0 (the words ks_inner gives with rot_c0); the digit set D and c0 are
// read once for all the rotations.  For 1 to 3 digits (ks_inner_multi_ok).
bool ks_inner_multi_ok(const fr_ctx *c, int level);
void ks_inner_multi(const fr_ctx *c, u64 *U, size_t ub, const u64 *D, const unsigned char *const *ksk, const u64 *g,
                    int nrot, int level, int batch, size_t sd, size_t su, const u64 *c0, size_t c0_sd);
// out[b][p][e] = P in[b][p][e] on the limbs e <= level and 0 on the special
// limbs (a ciphertext at level `level` lifted to Q_l U P; out items so words
// apart, polynomials nE limbs apart; in items si words apart)
void scale_ext(const fr_ctx *c, u64 *out, const u64 *in, int level, int nb, size_t so, size_t si);
// t01 = (sum a0 b0, sum a0 b1 + a1 b0), t2 = sum a1 b1 over n ciphertext
// pairs (nl limbs per polynomial; t01 = [2][nl][N], t2 = [nl][N])
void tensor_sum(const fr_ctx *c, u64 *t01, u64 *t2, int nl, int n, const u64 *const *a, const u64 *const *b);
// giant steps of rotations per key-sum launch at this level (bounded so the
// 128-bit lazy sums cannot overflow)
int ks_inner_sum_chunk(const fr_ctx *c, int level);
// U{0,1} (+)= sum over nj rotations (keys ksk[j], Galois elements g[j]; their
// digits D + j sdj) of the key inner products, for `batch` items
void ks_inner_sum(const fr_ctx *c, u64 *U0, u64 *U1, const u64 *D, const unsigned char *const *ksk, const u64 *g, int nj,
                  size_t sdj, int level, bool accumulate, int batch, size_t sd, size_t su);
// out[b] (+)= sum_j sigma_{g_j}(in[b][j]) on nlimbs limbs of one polynomial;
// level >= 0: the limbs past it are the special primes (Q_level U P)
void automorph_sum(const fr_ctx *c, u64 *out, const u64 *in, const u64 *g, int nj, int nlimbs, int nb, size_t sob,
                   size_t sij, size_t sib, int level = -1, bool accumulate = true);
// Z[p][i] (i < level) for the merged ModDown + rescale of relinearised
// products: Xu holds the coefficient forms of U's limbs level..level+nP at
// their storage positions, Xd that of d's limb level; Xd null: U's limb
// level already holds d_l + P^-1 U_l, or (no_d) there is no d term
void relin_rescale_prep(const fr_ctx *c, u64 *Z, const u64 *Xu, const u64 *Xd, int level, int npoly, size_t sz,
                        size_t sxu, size_t sxd, bool no_d = false);
// exact residues mod the special primes of the centered integers (-Q_l/2,
// Q_l/2] given by their level+1 limbs (coefficient form): Xp[b][j][N] from
// X[b][level+1][N] (mixed-radix digits, no floating point)
int crt_extend(fr_ctx *c, u64 *Xp, const u64 *X, int level, int npoly, size_t sxp, size_t sx);
// U[p] limb level <- d[p] limb level + P^-1 U[p] limb level (eval domain;
// polynomials su / sd words apart)
void fold_top(const fr_ctx *c, u64 *U, const u64 *d, int level, int npoly, size_t su, size_t sd);
// v = FBC_{P->Q}(Upc) (coefficient form) into V[level+1][N]
void moddown_fbc(const fr_ctx *c, u64 *V, const u64 *Upc, int level, int npoly);
// out_i = (accumulate ? out_i : 0) + (U_i - V_i) P^-1   (eval domain)
void moddown_finish(const fr_ctx *c, u64 *out, const u64 *U, const u64 *V, int level, int npoly,
                    size_t so, size_t su, size_t sv, bool accumulate);
// rescale helpers: Y[p][i] = centered(x_p) mod q_i, i < level
void rescale_prep(const fr_ctx *c, u64 *Y, const u64 *xtop, int level, int npoly, size_t sy, size_t sx);
// out[p][i] = (in[p][i] - Y[p][i]) q_level^-1
void rescale_finish(const fr_ctx *c, u64 *out, const u64 *in, const u64 *Y, int level, int npoly,
                    size_t so, size_t si, size_t sy);
// the hoisted product's MAC with its baby steps i >= 1 formed inside it
// from the ModUp digit set D (items sd words apart), c0 (queries C, sc
// words apart, [2][level+1][N]) and the keys ksk[i] / Galois elements g[i]
// (i = 1 .. n1-1); baby step 0 (P times the query) from C.  Outputs as
// bsgs_mac over Q_level U P (nE limbs).  Only where bsgs_ksmac_ok holds:
// n1 <= 32, ell = 16 n1, at most 3 digits, keys packed like the diagonals.
bool bsgs_ksmac_ok(const fr_ctx *c, int level, int n1, int ell, const DbLayout &lay);
void bsgs_ksmac(const fr_ctx *c, u64 *P, size_t pq, int nq, int n1,
                const unsigned char *const *diag, size_t dstride, const DbLayout &lay, const u64 *D, size_t sd,
                const u64 *C, size_t sc, const unsigned char *const *ksk, const u64 *g, int level);
// fused plaintext-diagonal multiply-accumulate of all giant steps for nq
// queries: baby[q * n1 + i] is baby step i of query q, diag[q] the diagonal
// group it is scored against (queries sharing a group should be adjacent);
// the n2 outputs of query q start at P + q * pq
// Limbs m > lq use the modulus m + pofs (a product over Q_lq U P with the
// special primes stored after limb lq).
void bsgs_mac(const fr_ctx *c, u64 *P, size_t pq, const u64 *const *baby, int nq, int n1,
              const unsigned char *const *diag, size_t dstride, const DbLayout &lay, int ell, int level,
              int baby_level, int lq = 1 << 30, int pofs = 0);
// diagonals between 64-bit limbs and the packed byte layout: nd diagonals,
// nl limbs each, src / dst nl N words apart on the 64-bit side
void db_pack(const fr_ctx *c, unsigned char *dst, size_t dstride, const DbLayout &lay, const u64 *src, int nl, int nd);
void db_unpack(const fr_ctx *c, u64 *dst, const unsigned char *src, size_t sstride, const DbLayout &lay, int nl,
               int nd);
// key-switching key blocks between 64-bit limbs ([nb][nmod][N]) and the
// KeyLayout bytes (nb blocks, KeyLayout::block bytes apart)
void key_pack(const fr_ctx *c, unsigned char *dst, const u64 *src, int nb);
void key_unpack(const fr_ctx *c, u64 *dst, const unsigned char *src, int nb);
// batched element-wise helpers (items addressed by pointer)
// out[b] = sum_t k[b][t] * src[b][t] over the first nl limbs of both
// polynomials of every source; out items contiguous [B][2][nl][N]
void scalar_batch(const fr_ctx *c, u64 *out, int nl, int B, const ScalarItem *items);
// out[b][q] = sum_s K[b][s] src[q][s] (src [nq][ns] pointers, sources of
// lp1[s] limbs per polynomial; K [nb][ns] small signed integers) on the
// first nl limbs of both polynomials, output (b, q) at out + b ob + q oq;
// each source read once for all outputs.  False (nothing launched) beyond
// 16 outputs, 16 sources or 8 queries.
bool scalar_mat(const fr_ctx *c, u64 *out, int nl, int nb, int nq, const u64 *const *src, const int *lp1, int ns,
                const long long *K, size_t ob, size_t oq);
// c0 limbs of item b (items `item` words apart) += v[b]
void add_const_batch(const fr_ctx *c, u64 *data, int nl, int B, const long long *v, size_t item);
// out[b] = a[b] + b[b] (op 0), a[b] - b[b] (op 1) or 2 a[b] - b[b] (op 2),
// + cst[b] on c0
void pair_batch(const fr_ctx *c, int nl, int B, const u64 *const *a, const u64 *const *b, u64 *const *out,
                const long long *cst, const int *op);
// tensor of B pairs: d0, d1 -> t01 + b * 2 lw, d2 -> t2 + b * lw
void tensor_batch(const fr_ctx *c, u64 *t01, u64 *t2, int nl, int B, const u64 *const *a, const u64 *const *b);
// rotation outputs of nitems ciphertexts by one Galois element g (U, V:
// consecutive items): out[b] = ModDown-finish(U_b, V_b) + (sigma_g(in[b].c0), 0)
void moddown_rot(const fr_ctx *c, u64 *const *out, const u64 *U, const u64 *V, const u64 *const *in, u64 g,
                 int level, int nitems);
// key generation / encryption / decryption combiners (eval domain)
void key_combine(const fr_ctx *c, u64 *b, const u64 *a, const u64 *e, const u64 *s_mont, const u64 *sp, int dlo,
                 int dhi, int nlimbs);
void encrypt_combine(const fr_ctx *c, u64 *c0, u64 *c1, const u64 *v, const u64 *e0, const u64 *e1, const u64 *msg,
                     const u64 *pkb, const u64 *pka, int nlimbs);
void decrypt_combine(const fr_ctx *c, u64 *out, const u64 *c0, const u64 *c1, const u64 *s_mont, int nlimbs);

// randomness
void sample_uniform(const fr_ctx *c, u64 *out, u64 seed, u64 poly, const LimbMap &map, int nlimbs);
// signed small polynomial (ternary or Gaussian) to residues on every limb
void sample_small(const fr_ctx *c, u64 *out, u64 seed, u64 poly, int kind, const LimbMap &map, int nlimbs);

// encoding
void encode_slots(const fr_ctx *c, u64 *out, const double *z, int n, int level, double scale, int batch,
                  size_t zstride, size_t ostride, double *work);
void decode_slots(const fr_ctx *c, double *z, const u64 *m_coeff, int level, double scale, double *work);
// database slot vectors for diagonals [d0, d0 + nd) of group g
void db_slots(const fr_ctx *c, double *out, const float *T, int K, int ell, int B, int n1, int g, int d0,
              int nd);
}  // namespace frk

// error helpers (api.cpp)
int fr_fail(int code, const char *fmt, ...);

#define FR_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) return fr_fail(FR_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)
