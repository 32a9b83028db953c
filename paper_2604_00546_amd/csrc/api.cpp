// api.cpp -- the C ABI of include/fr.h: context tables, keys, encoding,
// encryption, and the operation sequences of the hot path, each a short
// chain of kernel launches on the context's stream.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>

#include "fr_core.h"

using namespace frh;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512];

int fr_fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

extern "C" const char *fr_last_error(void) { return g_err; }

// An entry point abandoned because the device scratch could not grow: the
// work already queued (on the caller's and the auxiliary streams) finishes
// before the call returns, so the caller may free or reuse its buffers.
static int arena_full(fr_ctx *c, const ArenaFull &e) {
    if (c) {
        for (auto &a : c->aux)
            if (a) (void)hipStreamSynchronize(a);
        (void)hipStreamSynchronize(c->stream);
    }
    return fr_fail(FR_ENOMEM, "device scratch exhausted: %zu more bytes needed, %zu allocated, limit %zu", e.bytes,
                   e.allocated, e.limit);
}
#define FR_CATCH(ctx)                                                                 \
    catch (const ArenaFull &e_) {                                                     \
        return arena_full(ctx, e_);                                                   \
    }                                                                                 \
    catch (const std::bad_alloc &) {                                                  \
        return fr_fail(FR_ENOMEM, "host allocation failed");                         \
    }

#define CHECK(cond, code, ...) \
    do {                       \
        if (!(cond)) return fr_fail(code, __VA_ARGS__); \
    } while (0)

// stream ids of the key material and of an encryption (one Philox stream
// per polynomial: counter (index, limb, poly, 0), key (seed, domain))
static const u64 POLY_SECRET = 1, POLY_PK_A = 2, POLY_PK_E = 3;
static const u64 POLY_ENC_V = 0x2000001, POLY_ENC_E0 = 0x2000002, POLY_ENC_E1 = 0x2000003;
static u64 poly_ksk(u64 kid, int t) { return 0x1000000ull + kid * 16ull + (u64)t; }
static const int KIND_TERNARY = 2, KIND_GAUSS = 3;

// ---------------------------------------------------------------------------
// arena
// ---------------------------------------------------------------------------
void *Arena::get(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto &ch : chunks) {
        if (ch.size - ch.used >= bytes) {
            void *p = ch.base + ch.used;
            ch.used += bytes;
            return p;
        }
    }
    const size_t have = allocated();
    if (have > limit || limit - have < bytes) return nullptr;
    const size_t sz = std::min(std::max(bytes, (size_t)256 << 20), limit - have);
    char *b = nullptr;
    if (hipMalloc(&b, sz) != hipSuccess) {
        (void)hipGetLastError();  // clear the sticky allocation error
        return nullptr;
    }
    chunks.push_back({b, sz, bytes});
    return b;
}
bool Arena::grow(size_t bytes) {
    const size_t have = allocated();
    if (have > limit || limit - have < bytes) return false;
    char *b = nullptr;
    if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    chunks.push_back({b, bytes, 0});
    return true;
}
size_t Arena::allocated() const {
    size_t t = 0;
    for (auto &ch : chunks) t += ch.size;
    return t;
}
void Arena::reset() {
    size_t used = 0;
    for (auto &ch : chunks) {
        used += ch.used;
        ch.used = 0;
    }
    peak = std::max(peak, used);
}
void Arena::release() {
    for (auto &ch : chunks) (void)hipFree(ch.base);
    chunks.clear();
}

// ---------------------------------------------------------------------------
// fixed scratch of the allocation-free hoisted rotation
// ---------------------------------------------------------------------------
// One array per GPU, created with the code object and held until the process
// ends.  Host code never passes the symbol itself to a kernel (on the host it
// only stands in for the device array): the device address comes from
// hipGetSymbolAddress, once per device, in fr_ctx_create.
static __device__ __align__(256) unsigned char g_noalloc_scratch[FR_NOALLOC_SCRATCH_BYTES];
static const int kMaxDevices = 64;
static void *g_noalloc_addr[kMaxDevices];
static std::mutex g_noalloc_mu;

// the array's address on the current device (nullptr and a message on failure)
static void *noalloc_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_noalloc_scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_noalloc_addr[dev] = ptr;
    }
    return g_noalloc_addr[dev];
}

namespace {

// RAII scope: everything taken from the arena inside is given back at exit
// (stream order makes reuse by later launches safe).
struct Scope {
    Arena &a;
    std::vector<size_t> used;
    explicit Scope(Arena &ar) : a(ar) {
        for (auto &ch : a.chunks) used.push_back(ch.used);
    }
    ~Scope() {
        size_t tot = 0;
        for (auto &ch : a.chunks) tot += ch.used;
        a.peak = std::max(a.peak, tot);
        if (a.hold) return;  // space handed out while held stays taken
        for (size_t i = 0; i < a.chunks.size(); ++i) a.chunks[i].used = i < used.size() ? used[i] : 0;
    }
};

inline LimbMap qmap() { return LimbMap{0, INT_MAX, 0, INT_MAX, 0}; }
inline LimbMap allmap(const fr_ctx *c) { return LimbMap{0, INT_MAX, 0, c->nmod, 0}; }
inline LimbMap pmap(const fr_ctx *c) { return LimbMap{0, INT_MAX, 0, 0, c->L + 1}; }
inline LimbMap single(int mod) { return LimbMap{0, INT_MAX, 0, 0, mod}; }

// device scratch from the arena; when the arena cannot grow (device memory
// or the context's scratch limit) the call is abandoned with ArenaFull,
// which every entry point turns into FR_ENOMEM, so no kernel is ever given
// a null pointer
u64 *scratch(fr_ctx *c, size_t words) {
    const size_t bytes = std::max<size_t>(words, 1) * 8;
    void *p = c->arena.get(bytes);
    if (!p) throw ArenaFull{bytes, c->arena.allocated(), c->arena.limit};
    return (u64 *)p;
}

// internal ciphertext view
struct Ct {
    u64 *d;
    int level;
    double scale;
    u64 *c0() const { return d; }
    u64 *c1(const fr_ctx *c) const { return d + (size_t)(level + 1) * c->N; }
};

int check_ct(const fr_ctx *c, const fr_ct *x, const char *what) {
    CHECK(x && x->data, FR_EINVAL, "%s: null ciphertext", what);
    CHECK(x->level >= 0 && x->level <= c->L && x->level <= x->cap, FR_EINVAL, "%s: bad level %d (cap %d)", what,
          x->level, x->cap);
    return FR_OK;
}
int check_out(const fr_ctx *c, const fr_ct *x, int level, const char *what) {
    CHECK(x && x->data, FR_EINVAL, "%s: null output", what);
    CHECK(level >= 0 && level <= x->cap && level <= c->L, FR_EINVAL, "%s: output level %d exceeds capacity %d", what,
          level, x->cap);
    return FR_OK;
}

// keys and databases serve every context of their parameter set on the
// device (several contexts, each on its own stream, can share them)
bool same_params(const fr_ctx *a, const fr_ctx *b) {
    return a == b || (a->N == b->N && a->L == b->L && a->nP == b->nP && a->dnum == b->dnum &&
                      std::memcmp(a->mod, b->mod, sizeof(u64) * a->nmod) == 0);
}
int keys_ok(const fr_ctx *c, const fr_keys *K, const char *what) {
    CHECK(c && K, FR_EINVAL, "%s: null argument", what);
    CHECK(same_params(c, K->ctx), FR_EINVAL, "%s: keys of another parameter set", what);
    return FR_OK;
}
int db_ok(const fr_ctx *c, const fr_db *db, const char *what) {
    CHECK(c && db, FR_EINVAL, "%s: null argument", what);
    CHECK(same_params(c, db->ctx), FR_EINVAL, "%s: database of another parameter set", what);
    return FR_OK;
}

// calls that wait for the device or move data to or from the host cannot be
// recorded into a graph: refused while a capture is in progress
int no_capture(const fr_ctx *c, const char *what) {
    CHECK(!c->capturing, FR_EINVAL, "%s: not allowed while a graph capture is in progress", what);
    return FR_OK;
}

int flag_check(fr_ctx *c, const char *what) {
    int h = 0;
    FR_HIP(hipMemcpyAsync(&h, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    FR_HIP(hipStreamSynchronize(c->stream));
    if (h) {
        FR_HIP(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
        return fr_fail(FR_ERANGE, "%s: value out of the representable range (flag %d)", what, h);
    }
    return FR_OK;
}

// ---------------------------------------------------------------------------
// key switching pieces
// ---------------------------------------------------------------------------
// D[b][t] (b < batch, t < ndig) = ModUp of digit t of c1[b] (eval domain,
// c1 polynomials c1_stride words apart) over Q_level U P; D items are
// ndig * nE * N words apart.

void ks_modup(fr_ctx *c, const u64 *c1, int level, u64 *D, int batch = 1, size_t c1_stride = 0) {
    const int N = c->N, nE = level + 1 + c->nP, ndig = num_digits(c, level);
    const size_t lw = (size_t)(level + 1) * N, dstride = (size_t)ndig * nE * N;
    u64 *X = scratch(c, (size_t)batch * lw);
    frk::ntt_inv(c, X, level + 1, qmap(), batch, lw, c1, c1_stride);
    // items x digits up to which ModUp runs as one conversion launch and one
    // transform over all extended limbs (a tuning knob)
    if (batch * ndig <= c->tune[FR_TUNE_MODUP_MERGE]) {
        // small batches: every digit in one conversion launch and one
        // transform; the conversion copies each digit's own limbs in
        // evaluation form and the transform leaves them alone (where the
        // transform cannot, it re-derives them from coefficient form)
        const bool own = frk::ntt_own_skip_ok(c);
        frk::modup_all(c, D, X, level, batch, dstride, lw, own ? c1 : nullptr, c1_stride);
        LimbMap ext{0, INT_MAX, 0, level + 1, c->L + 1};
        frk::ntt_fwd(c, D, nE, ext, ndig * batch, (size_t)nE * N, nullptr, 0, own ? c->alpha : 0, ndig, level + 1);
        return;
    }
    // large batches: per digit, transforming only the converted limbs (the
    // conversion launch also copies the digit's own evaluation-form limbs).  The digits are
    // independent: outside a region that already spreads work over the
    // auxiliary streams, digit t > 0 runs on one of them
    const hipStream_t main_stream = c->stream;
    StreamRestore restore(c->stream);
    const int naux = c->arena.hold ? 0 : std::min(ndig - 1, fr_ctx::kAux);
    if (naux > 0) {
        (void)hipEventRecord(c->ev_fork, main_stream);
        for (int a = 0; a < naux; ++a) (void)hipStreamWaitEvent(c->aux[a], c->ev_fork, 0);
    }
    for (int t = 0; t < ndig; ++t) {
        c->stream = (naux > 0 && t > 0) ? c->aux[(t - 1) % naux] : main_stream;
        u64 *Dt = D + (size_t)t * nE * N;
        const int lo = t * c->alpha, nd = std::min(c->alpha, level + 1 - lo);
        frk::modup_digit(c, Dt, X, level, t, batch, dstride, lw, c1, c1_stride);
        LimbMap m{0, lo, nd, level + 1, c->L + 1};
        frk::ntt_fwd(c, Dt, nE - nd, m, batch, dstride);
    }
    c->stream = main_stream;
    for (int a = 0; a < naux; ++a) {
        (void)hipEventRecord(c->ev_join[a], c->aux[a]);
        (void)hipStreamWaitEvent(main_stream, c->ev_join[a], 0);
    }
}

// V[b] = the eval-domain ModDown correction of U[b] (b < nblk): iNTT of the
// P limbs, centered base conversion to Q_level, NTT.  U is [nblk][2][nE][N],
// V is [nblk][2][level+1][N].
void ks_moddown_prep(fr_ctx *c, const u64 *U, int nblk, int level, u64 *V) {
    const int N = c->N, nE = level + 1 + c->nP, nP = c->nP;
    u64 *Upc = scratch(c, (size_t)2 * nblk * nP * N);
    frk::ntt_inv(c, Upc, nP, pmap(c), 2 * nblk, (size_t)nP * N, U + (size_t)(level + 1) * N, (size_t)nE * N);
    frk::moddown_fbc(c, V, Upc, level, 2 * nblk);
    frk::ntt_fwd(c, V, level + 1, qmap(), 2 * nblk, (size_t)(level + 1) * N);
}

// out[b] (ciphertexts [2][level+1][N], polynomials so words apart) (+)=
// ModDown(U[b]) for b < nblk, U = [nblk][2][nE][N]; the finish runs inside
// the last pass of the forward transform of the correction
void ks_moddown_into(fr_ctx *c, const u64 *U, int nblk, int level, u64 *out, size_t so, bool accumulate) {
    Scope sc(c->arena);
    const int N = c->N, nE = level + 1 + c->nP, nP = c->nP;
    const size_t lw = (size_t)(level + 1) * N;
    u64 *Upc = scratch(c, (size_t)2 * nblk * nP * N);
    frk::ntt_inv(c, Upc, nP, pmap(c), 2 * nblk, (size_t)nP * N, U + lw, (size_t)nE * N);
    u64 *V = scratch(c, (size_t)2 * nblk * lw);
    frk::moddown_fbc(c, V, Upc, level, 2 * nblk);
    if (frk::ntt_fwd_moddown(c, V, level, 2 * nblk, U, (size_t)nE * N, out, so, accumulate)) return;
    frk::ntt_fwd(c, V, level + 1, qmap(), 2 * nblk, lw);
    frk::moddown_finish(c, out, U, V, level, 2 * nblk, so, (size_t)nE * N, lw, accumulate);
}

// out (ciphertext [2][level+1][N]) (+)= ModDown(U), U = [2][nE][N]
void ks_moddown(fr_ctx *c, const u64 *U, int level, u64 *out, bool accumulate) {
    ks_moddown_into(c, U, 1, level, out, (size_t)(level + 1) * c->N, accumulate);
}

// out = Rescale(in) for ncts consecutive ciphertexts at level l >= 1 (in:
// [ncts][2][l+1][N], out: [ncts][2][l][N]); out != in
void rescale_dev(fr_ctx *c, const u64 *in, int l, u64 *out, int ncts = 1) {
    Scope sc(c->arena);
    const int N = c->N, np = 2 * ncts;
    u64 *xt = scratch(c, (size_t)np * N);
    frk::ntt_inv(c, xt, 1, single(l), np, (size_t)N, in + (size_t)l * N, (size_t)(l + 1) * N);
    u64 *Y = scratch(c, (size_t)np * l * N);
    if (frk::ntt_fwd_rescale(c, Y, l, np, xt, in, (size_t)(l + 1) * N, out, (size_t)l * N)) return;
    frk::rescale_prep(c, Y, xt, l, np, (size_t)l * N, (size_t)N);
    frk::ntt_fwd(c, Y, l, qmap(), np, (size_t)l * N);
    frk::rescale_finish(c, out, in, Y, l, np, (size_t)l * N, (size_t)(l + 1) * N, (size_t)l * N);
}

// out (B items [2][l][N]) = Rescale(d + ModDown(U)) for relinearised
// products at level l >= 1 (d = the tensor's first two polynomials, B items
// [2][l+1][N]; U = [B][2][nE][N]).  On the radix-16 rings the ModDown and
// the rescale share one forward transform of l limbs; otherwise they run in
// sequence (d is then overwritten).
// true when relin_rescale_into takes U with its top limb folded by ks_inner
bool relin_folds(const fr_ctx *c) { return c->logN == 16 || c->logN == 12; }

void relin_rescale_into(fr_ctx *c, u64 *d, const u64 *U, int B, int l, u64 *out) {
    Scope sc(c->arena);
    const int N = c->N, nE = l + 1 + c->nP, np = 2 * B;
    const size_t lw = (size_t)(l + 1) * N;
    if (relin_folds(c)) {
        // U's limb l holds d_l + P^-1 U_l: one inverse transform of it and
        // the P limbs gives everything the merged step needs
        u64 *Xu = scratch(c, (size_t)np * nE * N);
        LimbMap top_and_p{l, INT_MAX, 0, l + 1, c->L + 1};
        frk::ntt_inv(c, Xu, c->nP + 1, top_and_p, np, (size_t)nE * N, U, (size_t)nE * N);
        u64 *Z = scratch(c, (size_t)np * l * N);
        frk::relin_rescale_prep(c, Z, Xu, nullptr, l, np, (size_t)l * N, (size_t)nE * N, 0);
        frk::ntt_fwd_relin_rescale(c, Z, l, np, U, (size_t)nE * N, d, lw, out, (size_t)l * N);
        return;
    }
    ks_moddown_into(c, U, B, l, d, lw, true);
    rescale_dev(c, d, l, out, B);
}
// d = relinearise + rescale of a x b (both at level l) into out at l - 1
int mul_relin_rescale_dev(fr_ctx *c, const fr_keys *K, const Ct &a, const Ct &b, u64 *out) {
    const KeyEntry *rk = K->find(0);
    CHECK(rk, FR_ENOKEY, "relinearisation key missing");
    Scope sc(c->arena);
    const int N = c->N, l = a.level, nE = l + 1 + c->nP;
    const size_t lw = (size_t)(l + 1) * N;
    u64 *T3 = scratch(c, 3 * lw);
    frk::tensor(c, T3, T3 + lw, T3 + 2 * lw, a.c0(), a.c1(c), b.c0(), b.c1(c), l + 1);
    u64 *D = scratch(c, (size_t)num_digits(c, l) * nE * N);
    ks_modup(c, T3 + 2 * lw, l, D);
    u64 *U = scratch(c, (size_t)2 * nE * N);
    frk::ks_inner(c, U, U + (size_t)nE * N, D, rk->data, 1, l, false, 1, 0, 0, relin_folds(c) ? T3 : nullptr, 0);
    relin_rescale_into(c, T3, U, 1, l, out);
    return FR_OK;
}

void residues_of(const fr_ctx *c, long long v, int nl, u64 *r, u64 *rsh) {
    for (int i = 0; i < nl; ++i) {
        const u64 q = c->mod[i];
        u64 x;
        if (v >= 0) x = (u64)v % q;
        else {
            u64 a = (u64)(-(v + 1)) % q;  // avoids overflow at LLONG_MIN
            a = (a + 1) % q;
            x = a ? q - a : 0;
        }
        r[i] = x;
        if (rsh) rsh[i] = shoup_companion(x, q);
    }
}

// out = k * a (every limb), a and out at the same level
void mul_int_dev(fr_ctx *c, const u64 *a, size_t sa, int nl, long long k, u64 *out, size_t so) {
    u64 r[FR_MAXMOD], rs[FR_MAXMOD];
    residues_of(c, k, nl, r, rs);
    frk::mul_const(c, out, a, r, rs, nl, 2, so, sa);
}

// c0 += round(cst * scale) as a constant polynomial (in place)
void add_const_dev(fr_ctx *c, u64 *c0, int level, double cst, double scale) {
    long long v = (long long)std::nearbyint(cst * scale);
    u64 r[FR_MAXMOD];
    residues_of(c, v, level + 1, r, nullptr);
    frk::add_const(c, c0, c0, r, level + 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
template <class T>
static int upload(T **dst, const std::vector<T> &src) {
    FR_HIP(hipMalloc(dst, std::max<size_t>(src.size(), 1) * sizeof(T)));
    FR_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return FR_OK;
}

// x 2^64 mod q: table entries that multiply 128-bit lazy sums, so that one
// Montgomery reduction of the sum yields the canonical residue
static u64 to_mont(u64 x, u64 q) { return (u64)(((unsigned __int128)x << 64) % q); }

static u64 prod_mod(const fr_ctx *c, const std::vector<int> &idx, int skip, u64 r) {
    u64 p = 1 % r;
    for (int i : idx)
        if (i != skip) p = mulmod_h(p, c->mod[i] % r, r);
    return p;
}

static int ctx_build(fr_ctx *c) {
    const int N = c->N, nm = c->nmod, L = c->L, nP = c->nP;
    // per-modulus constants and twiddles
    std::vector<ModConst> mc(nm);
    std::vector<u64> tw((size_t)nm * N), tws((size_t)nm * N), itw((size_t)nm * N), itws((size_t)nm * N);
    for (int m = 0; m < nm; ++m) {
        const u64 q = c->mod[m];
        mc[m] = make_modconst(q, N);
        c->hmod[m] = mc[m];
        const u64 psi = primitive_2n_root(q, N), ipsi = invmod_h(psi, q);
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; ++k) {
            pw[k] = mulmod_h(pw[k - 1], psi, q);
            ipw[k] = mulmod_h(ipw[k - 1], ipsi, q);
        }
        for (int k = 0; k < N; ++k) {
            u32 r = 0, x = (u32)k;
            for (int b = 0; b < c->logN; ++b) {
                r = (r << 1) | (x & 1);
                x >>= 1;
            }
            const size_t o = (size_t)m * N + k;
            tw[o] = pw[r];
            tws[o] = shoup_companion(tw[o], q);
            itw[o] = ipw[r];
            itws[o] = shoup_companion(itw[o], q);
        }
    }
    if (int e = upload(&c->d_mod, mc)) return e;
    if (int e = upload(&c->d_tw, tw)) return e;
    if (int e = upload(&c->d_tw_sh, tws)) return e;
    if (int e = upload(&c->d_itw, itw)) return e;
    if (int e = upload(&c->d_itw_sh, itws)) return e;
    {
        std::vector<u64> t2((size_t)2 * nm * N), it2((size_t)2 * nm * N);
        for (size_t o = 0; o < (size_t)nm * N; ++o) {
            t2[2 * o] = tw[o];
            t2[2 * o + 1] = tws[o];
            it2[2 * o] = itw[o];
            it2[2 * o + 1] = itws[o];
        }
        if (int e = upload(&c->d_tw2, t2)) return e;
        if (int e = upload(&c->d_itw2, it2)) return e;
    }

    // ModUp tables
    std::vector<u64> mu;
    for (int l = 0; l <= L; ++l) {
        const int nE = l + 1 + nP, ndig = num_digits(c, l);
        for (int t = 0; t < ndig; ++t) {
            c->modup_off[l][t] = mu.size();
            const int lo = t * c->alpha, nd = std::min(c->alpha, l + 1 - lo);
            std::vector<int> dig;
            for (int d = 0; d < nd; ++d) dig.push_back(lo + d);
            for (int d = 0; d < nd; ++d) {
                const u64 qi = c->mod[lo + d];
                const u64 inv = invmod_h(prod_mod(c, dig, lo + d, qi), qi);
                mu.push_back(inv);
            }
            for (int d = 0; d < nd; ++d) mu.push_back(shoup_companion(mu[c->modup_off[l][t] + d], c->mod[lo + d]));
            for (int e = 0; e < nE; ++e) {
                const int gm = e <= l ? e : L + 1 + (e - l - 1);
                for (int d = 0; d < nd; ++d) mu.push_back(to_mont(prod_mod(c, dig, lo + d, c->mod[gm]), c->mod[gm]));
            }
        }
    }
    if (int e = upload(&c->d_modup, mu)) return e;

    // ModDown tables
    std::vector<u64> md;
    std::vector<int> pidx;
    for (int j = 0; j < nP; ++j) pidx.push_back(L + 1 + j);
    for (int j = 0; j < nP; ++j) md.push_back(invmod_h(prod_mod(c, pidx, L + 1 + j, c->mod[L + 1 + j]), c->mod[L + 1 + j]));
    for (int j = 0; j < nP; ++j) md.push_back(shoup_companion(md[j], c->mod[L + 1 + j]));
    for (int i = 0; i <= L; ++i)
        for (int j = 0; j < nP; ++j) md.push_back(to_mont(prod_mod(c, pidx, L + 1 + j, c->mod[i]), c->mod[i]));
    std::vector<u64> pinv(L + 1), pinvs(L + 1);
    for (int i = 0; i <= L; ++i) {
        const u64 pm = prod_mod(c, pidx, -1, c->mod[i]);
        c->P_mod_q[i] = pm;
        c->P_mod_q_sh[i] = shoup_companion(pm, c->mod[i]);
        pinv[i] = invmod_h(pm, c->mod[i]);
        pinvs[i] = shoup_companion(pinv[i], c->mod[i]);
        c->P_inv_q[i] = pinv[i];
        c->P_inv_q_sh[i] = pinvs[i];
    }
    md.insert(md.end(), pinv.begin(), pinv.end());
    md.insert(md.end(), pinvs.begin(), pinvs.end());
    for (int i = 0; i <= L; ++i) md.push_back(c->P_mod_q[i]);
    for (int j = 0; j < nP; ++j) {
        const double inv = 1.0 / (double)c->mod[L + 1 + j];
        u64 bits;
        std::memcpy(&bits, &inv, 8);
        md.push_back(bits);
    }
    // [i][e] = -e P 2^64 mod q_i, e = 0..nP: the overflow correction in the
    // Montgomery domain of the conversion's 128-bit sums
    for (int i = 0; i <= L; ++i)
        for (int e = 0; e <= nP; ++e) {
            const u64 qi = c->mod[i];
            const u64 eP = mulmod_h((u64)e, c->P_mod_q[i], qi);
            md.push_back(to_mont(eP ? qi - eP : 0, qi));
        }
    // [i] = P 2^64 mod q_i: P times a word inside a Montgomery-reduced sum
    for (int i = 0; i <= L; ++i) md.push_back(to_mont(c->P_mod_q[i], c->mod[i]));
    if (int e = upload(&c->d_moddown, md)) return e;
    {  // Phat_j and P as multiword integers (ModDown's exact overflow decision)
        std::vector<u64> pb((size_t)kPbigRows * kPbigWords, 0);
        auto mul_small = [](u64 *w, u64 m) {
            u64 carry = 0;
            for (int k = 0; k < kPbigWords; ++k) {
                const unsigned __int128 t = (unsigned __int128)w[k] * m + carry;
                w[k] = (u64)t;
                carry = (u64)(t >> 64);
            }
        };
        u64 *Pw = pb.data() + (size_t)(kPbigRows - 1) * kPbigWords;
        Pw[0] = 1;
        for (int j = 0; j < nP; ++j) {
            u64 *row = pb.data() + (size_t)j * kPbigWords;
            row[0] = 1;
            for (int jj = 0; jj < nP; ++jj)
                if (jj != j) mul_small(row, c->mod[L + 1 + jj]);
            mul_small(Pw, c->mod[L + 1 + j]);
        }
        if (int e = upload(&c->d_pbig, pb)) return e;
    }

    // rescale tables: q_l^-1 mod q_i, then (P q_l)^-1 mod q_i (ModDown and
    // rescale in one product), each [L+1][value, companion][L+1]
    const size_t rtab = (size_t)(L + 1) * (L + 1) * 2;
    std::vector<u64> rs(2 * rtab, 0);
    for (int l = 1; l <= L; ++l)
        for (int i = 0; i < l; ++i) {
            const u64 qi = c->mod[i];
            const u64 v = invmod_h(c->mod[l] % qi, qi);
            rs[(size_t)l * (L + 1) * 2 + i] = v;
            rs[(size_t)l * (L + 1) * 2 + (L + 1) + i] = shoup_companion(v, qi);
            const u64 w = mulmod_h(v, c->P_inv_q[i], qi);
            rs[rtab + (size_t)l * (L + 1) * 2 + i] = w;
            rs[rtab + (size_t)l * (L + 1) * 2 + (L + 1) + i] = shoup_companion(w, qi);
        }
    if (int e = upload(&c->d_rescale, rs)) return e;

    // CRT lift tables
    const int W = 4 * (L + 1) + 1;
    std::vector<u64> crt((size_t)(L + 1) * W, 0);
    for (int l = 0; l <= L; ++l) {
        u64 *t = crt.data() + (size_t)l * W;
        std::vector<int> qs;
        for (int i = 0; i <= l; ++i) qs.push_back(i);
        u64 Q64 = 1;
        for (int i = 0; i <= l; ++i) Q64 *= c->mod[i];
        for (int i = 0; i <= l; ++i) {
            const u64 qi = c->mod[i];
            t[i] = invmod_h(prod_mod(c, qs, i, qi), qi);
            t[(L + 1) + i] = shoup_companion(t[i], qi);
            u64 h64 = 1;
            for (int j = 0; j <= l; ++j)
                if (j != i) h64 *= c->mod[j];
            t[2 * (L + 1) + i] = h64;
            double inv = 1.0 / (double)qi;
            std::memcpy(&t[3 * (L + 1) + i], &inv, 8);
        }
        t[4 * (L + 1)] = Q64;
    }
    if (int e = upload(&c->d_crt, crt)) return e;

    // FFT tables
    std::vector<double> fw((size_t)N), zt((size_t)2 * N);
    for (int k = 0; k < N / 2; ++k) {
        const double a = 2.0 * M_PI * (double)k / (double)N;
        fw[2 * k] = std::cos(a);
        fw[2 * k + 1] = -std::sin(a);
    }
    for (int k = 0; k < N; ++k) {
        const double a = M_PI * (double)k / (double)N;
        zt[2 * k] = std::cos(a);
        zt[2 * k + 1] = std::sin(a);
    }
    std::vector<u32> sp(N / 2);
    u64 e5 = 1;
    for (int j = 0; j < N / 2; ++j) {
        sp[j] = (u32)((e5 - 1) / 2);
        e5 = (e5 * 5) % (2ull * N);
    }
    if (int e = upload(&c->d_fft_w, fw)) return e;
    if (int e = upload(&c->d_zeta, zt)) return e;
    if (int e = upload(&c->d_slot_pos, sp)) return e;
    gauss_cdt(c->cdt);
    FR_HIP(hipMalloc(&c->d_flag, sizeof(int)));
    FR_HIP(hipMemset(c->d_flag, 0, sizeof(int)));
    return FR_OK;
}

extern "C" int fr_ctx_create(const fr_params *p, fr_ctx **out) {
    CHECK(p && out, FR_EINVAL, "fr_ctx_create: null argument");
    CHECK(p->log_n >= 10 && p->log_n <= 16, FR_EINVAL, "fr_ctx_create: log_n must be in [10, 16]");
    CHECK(p->n_mid >= 0 && p->n_special >= 1 && p->dnum >= 1 && 1 + p->n_mid + p->n_special <= FR_MAXMOD &&
              p->n_mid + 1 <= FR_MAXLEVEL,
          FR_EINVAL, "fr_ctx_create: bad prime counts");
    CHECK(p->q0_bits >= 30 && p->q0_bits <= 60 && p->mid_bits >= 30 && p->mid_bits <= 60 && p->special_bits >= 30 &&
              p->special_bits <= 60,
          FR_EINVAL, "fr_ctx_create: prime sizes must be 30..60 bits");
    const int alpha = (p->n_mid + 1 + p->dnum - 1) / p->dnum;
    CHECK(alpha <= 8 && p->n_special <= 8 && p->dnum <= 8, FR_EINVAL,
          "fr_ctx_create: digit size and special primes limited to 8");
    fr_ctx *c = new fr_ctx();
    c->logN = p->log_n;
    c->N = 1 << p->log_n;
    c->L = p->n_mid;
    c->nP = p->n_special;
    c->dnum = p->dnum;
    c->alpha = alpha;
    c->nmod = c->L + 1 + c->nP;
    if (choose_primes(c->logN, p->q0_bits, p->n_mid, p->mid_bits, p->n_special, p->special_bits, c->mod) != c->nmod) {
        delete c;
        return fr_fail(FR_EINVAL, "fr_ctx_create: not enough primes of the requested sizes");
    }
    {  // key-switching key storage: limbs of moduli below 2^40 in 5 bytes per word
        size_t o = 0;
        for (int m = 0; m < c->nmod; ++m) {
            c->klay.packed[m] = c->mod[m] < (1ull << 40);
            c->klay.off[m] = (unsigned)o;
            o += (c->klay.packed[m] ? 5 : 8) * (size_t)c->N;
        }
        c->klay.block = o;
    }
    int e = ctx_build(c);
    if (!e) {  // the allocation-free rotation's scratch: a one-chunk arena over this device's array
        void *fixed = noalloc_address();
        if (!fixed)
            e = fr_fail(FR_EHIP, "fr_ctx_create: no address for the fixed scratch array");
        else {
            c->fixed_arena.chunks.push_back({(char *)fixed, FR_NOALLOC_SCRATCH_BYTES, 0});
            c->fixed_arena.limit = FR_NOALLOC_SCRATCH_BYTES;
        }
    }
    for (int a = 0; !e && a < fr_ctx::kAux; ++a)
        if (hipStreamCreateWithFlags(&c->aux[a], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_join[a], hipEventDisableTiming) != hipSuccess)
            e = fr_fail(FR_EHIP, "fr_ctx_create: auxiliary stream");
    if (!e && hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess)
        e = fr_fail(FR_EHIP, "fr_ctx_create: event");
    for (int i = 0; !e && i < fr_ctx::kDagEv; ++i)
        if (hipEventCreateWithFlags(&c->ev_dag[i], hipEventDisableTiming) != hipSuccess)
            e = fr_fail(FR_EHIP, "fr_ctx_create: event");
    if (e) {
        fr_ctx_destroy(c);
        return e;
    }
    *out = c;
    return FR_OK;
}

extern "C" void fr_ctx_destroy(fr_ctx *c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)c->d_mod, (void *)c->d_tw, (void *)c->d_tw_sh, (void *)c->d_itw, (void *)c->d_itw_sh,
                    (void *)c->d_tw2, (void *)c->d_itw2,
                    (void *)c->d_modup, (void *)c->d_moddown, (void *)c->d_pbig, (void *)c->d_rescale, (void *)c->d_crt,
                    (void *)c->d_fft_w, (void *)c->d_zeta, (void *)c->d_slot_pos, (void *)c->d_flag})
        if (p) (void)hipFree(p);
    c->arena.release();
    for (int a = 0; a < fr_ctx::kAux; ++a)
        if (c->aux[a]) (void)hipStreamDestroy(c->aux[a]);
    for (int a = 0; a < fr_ctx::kAux; ++a)
        if (c->ev_join[a]) (void)hipEventDestroy(c->ev_join[a]);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (int i = 0; i < fr_ctx::kDagEv; ++i)
        if (c->ev_dag[i]) (void)hipEventDestroy(c->ev_dag[i]);
    if (c->prof) {
        for (auto &e : c->prof->ev) (void)hipEventDestroy(e);
        delete c->prof;
    }
    delete c;
}

extern "C" int fr_ctx_set_stream(fr_ctx *c, void *stream) try {
    CHECK(c, FR_EINVAL, "null context");
    CHECK(!c->capturing, FR_EINVAL, "fr_ctx_set_stream: a graph capture is in progress");
    if (c->stream != (hipStream_t)stream) FR_HIP(hipStreamSynchronize(c->stream));
    c->stream = (hipStream_t)stream;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_ctx_sync(fr_ctx *c) try {
    if (c) if (int e_ = no_capture(c, "fr_ctx_sync")) return e_;
    CHECK(c, FR_EINVAL, "null context");
    FR_HIP(hipStreamSynchronize(c->stream));
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_ctx_set_scratch_limit(fr_ctx *c, uint64_t bytes) try {
    CHECK(c, FR_EINVAL, "null context");
    c->arena.limit = bytes ? (size_t)bytes : ~(size_t)0;
    if (c->arena.allocated() > c->arena.limit) {
        CHECK(!c->capturing, FR_EINVAL, "fr_ctx_set_scratch_limit: a graph capture is in progress");
        FR_HIP(hipStreamSynchronize(c->stream));
        for (auto &a : c->aux) FR_HIP(hipStreamSynchronize(a));
        c->arena.release();
        ++c->arena_gen;
    }
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_ctx_set_tune(fr_ctx *c, int32_t knob, int32_t value) {
    CHECK(c, FR_EINVAL, "null context");
    CHECK(knob >= 0 && knob < FR_TUNE_COUNT, FR_EINVAL, "fr_ctx_set_tune: unknown knob %d", knob);
    static const int lo[FR_TUNE_COUNT] = {0, 0, 0, 0, 0, 1, 1, 0, 0, 0};
    static const int hi[FR_TUNE_COUNT] = {1 << 20, 1 << 20, 1 << 20, 1 << 20, 1 << 20, 16, 16, 1, 2, 1};
    CHECK(value >= lo[knob] && value <= hi[knob], FR_EINVAL, "fr_ctx_set_tune: knob %d takes %d..%d, not %d", knob,
          lo[knob], hi[knob], value);
    CHECK(!c->capturing, FR_EINVAL, "fr_ctx_set_tune: a graph capture is in progress");
    c->tune[knob] = value;
    return FR_OK;
}

extern "C" int fr_ctx_get_tune(const fr_ctx *c, int32_t knob, int32_t *value) {
    CHECK(c && value, FR_EINVAL, "fr_ctx_get_tune: null argument");
    CHECK(knob >= 0 && knob < FR_TUNE_COUNT, FR_EINVAL, "fr_ctx_get_tune: unknown knob %d", knob);
    *value = c->tune[knob];
    return FR_OK;
}

extern "C" int fr_ctx_scratch_info(const fr_ctx *c, uint64_t *allocated, uint64_t *peak) {
    CHECK(c, FR_EINVAL, "null context");
    if (allocated) *allocated = c->arena.allocated();
    if (peak) *peak = c->arena.peak;
    return FR_OK;
}

extern "C" int fr_ctx_reserve(fr_ctx *c, uint64_t bytes) try {
    if (c) if (int e_ = no_capture(c, "fr_ctx_reserve")) return e_;
    CHECK(c, FR_EINVAL, "null context");
    const size_t have = c->arena.allocated();
    if (have >= bytes) return FR_OK;
    CHECK(c->arena.grow((size_t)bytes - have), FR_ENOMEM,
          "fr_ctx_reserve: cannot grow the scratch to %llu bytes (limit %zu)", (unsigned long long)bytes,
          c->arena.limit);
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_ctx_dims(const fr_ctx *c, int32_t *n, int32_t *L, int32_t *ns, int32_t *alpha, int32_t *dnum) {
    CHECK(c, FR_EINVAL, "null context");
    if (n) *n = c->N;
    if (L) *L = c->L;
    if (ns) *ns = c->nP;
    if (alpha) *alpha = c->alpha;
    if (dnum) *dnum = c->dnum;
    return FR_OK;
}

extern "C" uint64_t fr_ctx_modulus(const fr_ctx *c, int32_t g) { return (c && g >= 0 && g < c->nmod) ? c->mod[g] : 0; }

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
extern "C" void fr_keys_destroy(fr_keys *k) {
    if (!k) return;
    (void)hipStreamSynchronize(k->ctx->stream);
    for (auto &e : k->ksk) (void)hipFree(e.data);
    (void)hipFree(k->s_eval);
    (void)hipFree(k->s_mont);
    (void)hipFree(k->pk);
    delete k;
}

extern "C" int fr_keygen(fr_ctx *c, uint64_t seed, const int32_t *rots, int32_t nrot, fr_keys **out) try {
    if (c) if (int e_ = no_capture(c, "fr_keygen")) return e_;
    CHECK(c && out && (nrot == 0 || rots), FR_EINVAL, "fr_keygen: null argument");
    c->arena.reset();
    Scope sc(c->arena);
    const int N = c->N, nm = c->nmod, L = c->L;
    const size_t lw = (size_t)N;
    std::unique_ptr<fr_keys, void (*)(fr_keys *)> K(new fr_keys(), fr_keys_destroy);
    K->ctx = c;
    FR_HIP(hipMalloc(&K->s_eval, nm * lw * 8));
    FR_HIP(hipMalloc(&K->s_mont, nm * lw * 8));
    FR_HIP(hipMalloc(&K->pk, 2 * (L + 1) * lw * 8));
    const LimbMap all = allmap(c);
    frk::sample_small(c, K->s_eval, seed, POLY_SECRET, KIND_TERNARY, all, nm);
    frk::ntt_fwd(c, K->s_eval, nm, all, 1, 0);
    FR_HIP(hipMemcpyAsync(K->s_mont, K->s_eval, nm * lw * 8, hipMemcpyDeviceToDevice, c->stream));
    frk::mont_scale(c, K->s_mont, nm, all, 1, 0, true);
    // public key
    u64 *e = scratch(c, nm * lw);
    CHECK(e, FR_ENOMEM, "fr_keygen: scratch");
    u64 *pka = K->pk + (size_t)(L + 1) * lw;
    frk::sample_uniform(c, pka, seed, POLY_PK_A, qmap(), L + 1);
    frk::ntt_fwd(c, pka, L + 1, qmap(), 1, 0);
    frk::sample_small(c, e, seed, POLY_PK_E, KIND_GAUSS, qmap(), L + 1);
    frk::ntt_fwd(c, e, L + 1, qmap(), 1, 0);
    frk::key_combine(c, K->pk, pka, e, K->s_mont, nullptr, 0, 0, L + 1);
    // key ids: s^2 (0) and the distinct Galois elements
    std::vector<u64> kids{0};
    for (int r = 0; r < nrot; ++r) {
        const u64 g = galois_element(N, rots[r]);
        if (g != 1 && std::find(kids.begin(), kids.end(), g) == kids.end()) kids.push_back(g);
    }
    u64 *sp = scratch(c, (size_t)(L + 1) * lw);
    // a key in 64-bit limbs [dnum][2][nm][N], packed into its KeyLayout blocks
    u64 *kt = scratch(c, (size_t)c->dnum * 2 * nm * lw);
    CHECK(sp && kt, FR_ENOMEM, "fr_keygen: scratch");
    for (u64 kid : kids) {
        KeyEntry ke{kid, nullptr};
        FR_HIP(hipMalloc(&ke.data, (size_t)c->dnum * 2 * c->klay.block));
        K->ksk.push_back(ke);
        if (kid == 0) frk::mul_pt(c, sp, K->s_eval, K->s_eval, L + 1, 1, 0, 0);
        else frk::automorph(c, sp, K->s_eval, kid, L + 1, 1, 0, 0, false);
        for (int t = 0; t < c->dnum; ++t) {
            u64 *b = kt + (size_t)(t * 2 + 0) * nm * lw;
            u64 *a = kt + (size_t)(t * 2 + 1) * nm * lw;
            frk::sample_uniform(c, a, seed, poly_ksk(kid, t), all, nm);
            frk::ntt_fwd(c, a, nm, all, 1, 0);
            frk::sample_small(c, e, seed, poly_ksk(kid, t), KIND_GAUSS, all, nm);
            frk::ntt_fwd(c, e, nm, all, 1, 0);
            const int dlo = t * c->alpha, dhi = std::min(dlo + c->alpha, L + 1);
            frk::key_combine(c, b, a, e, K->s_mont, sp, dlo, dhi, nm);
        }
        frk::mont_scale(c, kt, nm, all, 2 * c->dnum, (size_t)nm * lw, true);
        frk::key_pack(c, ke.data, kt, 2 * c->dnum);
    }
    FR_HIP(hipGetLastError());
    FR_HIP(hipStreamSynchronize(c->stream));
    *out = K.release();
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_keys_export(fr_ctx *c, const fr_keys *K, int32_t what, uint64_t kid, uint64_t *host) try {
    if (int e = keys_ok(c, K, "fr_keys_export")) return e;
    if (c) if (int e_ = no_capture(c, "fr_keys_export")) return e_;
    CHECK(c && K && host, FR_EINVAL, "fr_keys_export: null argument");
    c->arena.reset();
    Scope sc(c->arena);
    const int N = c->N, nm = c->nmod, L = c->L;
    if (what == 0) {
        u64 *t = scratch(c, N);
        FR_HIP(hipMemcpyAsync(t, K->s_eval, (size_t)N * 8, hipMemcpyDeviceToDevice, c->stream));
        frk::ntt_inv(c, t, 1, qmap(), 1, 0);
        std::vector<u64> h(N);
        FR_HIP(hipMemcpyAsync(h.data(), t, (size_t)N * 8, hipMemcpyDeviceToHost, c->stream));
        FR_HIP(hipStreamSynchronize(c->stream));
        int64_t *o = reinterpret_cast<int64_t *>(host);
        for (int k = 0; k < N; ++k) o[k] = h[k] == 0 ? 0 : (h[k] == 1 ? 1 : -1);
        return FR_OK;
    }
    if (what == 1) {
        const size_t w = (size_t)2 * (L + 1) * N;
        u64 *t = scratch(c, w);
        FR_HIP(hipMemcpyAsync(t, K->pk, w * 8, hipMemcpyDeviceToDevice, c->stream));
        frk::ntt_inv(c, t, L + 1, qmap(), 2, (size_t)(L + 1) * N);
        FR_HIP(hipMemcpyAsync(host, t, w * 8, hipMemcpyDeviceToHost, c->stream));
        FR_HIP(hipStreamSynchronize(c->stream));
        return FR_OK;
    }
    if (what == 2) {
        const KeyEntry *ke = K->find(kid);
        CHECK(ke, FR_ENOKEY, "fr_keys_export: no key for id %llu", (unsigned long long)kid);
        const size_t w = (size_t)c->dnum * 2 * nm * N;
        u64 *t = scratch(c, w);
        CHECK(t, FR_ENOMEM, "fr_keys_export: scratch");
        frk::key_unpack(c, t, ke->data, 2 * c->dnum);
        frk::mont_scale(c, t, nm, allmap(c), 2 * c->dnum, (size_t)nm * N, false);
        frk::ntt_inv(c, t, nm, allmap(c), 2 * c->dnum, (size_t)nm * N);
        FR_HIP(hipMemcpyAsync(host, t, w * 8, hipMemcpyDeviceToHost, c->stream));
        FR_HIP(hipStreamSynchronize(c->stream));
        return FR_OK;
    }
    return fr_fail(FR_EINVAL, "fr_keys_export: unknown selector %d", what);
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// encode / import / export / encrypt / decrypt / decode
// ---------------------------------------------------------------------------
static int encode_common(fr_ctx *c, const double *zdev, int n, int level, double scale, fr_pt *out) {
    const int N = c->N;
    double *work = (double *)c->arena.get((size_t)N * 16);
    CHECK(work, FR_ENOMEM, "fr_encode: scratch");
    frk::encode_slots(c, out->data, zdev, n, level, scale, 1, 0, 0, work);
    frk::ntt_fwd(c, out->data, level + 1, qmap(), 1, 0);
    if (int e = flag_check(c, "fr_encode")) return e;
    out->level = level;
    out->scale = scale;
    return FR_OK;
}

extern "C" int fr_encode(fr_ctx *c, const double *z, int32_t n, int32_t level, double scale, fr_pt *out) try {
    if (c) if (int e_ = no_capture(c, "fr_encode")) return e_;
    CHECK(c && out && out->data && (n == 0 || z), FR_EINVAL, "fr_encode: null argument");
    CHECK(n >= 0 && n <= c->N / 2 && level >= 0 && level <= c->L && level <= out->cap, FR_EINVAL,
          "fr_encode: bad size or level");
    c->arena.reset();
    Scope sc(c->arena);
    double *zd = (double *)c->arena.get((size_t)std::max(n, 1) * 8);
    CHECK(zd, FR_ENOMEM, "fr_encode: scratch");
    if (n) FR_HIP(hipMemcpyAsync(zd, z, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
    FR_HIP(hipStreamSynchronize(c->stream));
    return encode_common(c, zd, n, level, scale, out);
} FR_CATCH(c)

extern "C" int fr_encode_device(fr_ctx *c, const double *z, int32_t n, int32_t level, double scale, fr_pt *out) try {
    if (c) if (int e_ = no_capture(c, "fr_encode_device")) return e_;
    CHECK(c && out && out->data && (n == 0 || z), FR_EINVAL, "fr_encode_device: null argument");
    CHECK(n >= 0 && n <= c->N / 2 && level >= 0 && level <= c->L && level <= out->cap, FR_EINVAL,
          "fr_encode_device: bad size or level");
    c->arena.reset();
    Scope sc(c->arena);
    return encode_common(c, z, n, level, scale, out);
} FR_CATCH(c)

static int import_poly(fr_ctx *c, const uint64_t *host, int nl, int npoly, u64 *dst) {
    const size_t w = (size_t)npoly * nl * c->N;
    std::vector<u64> h(host, host + w);
    for (int p = 0; p < npoly; ++p)
        for (int i = 0; i < nl; ++i)
            for (int k = 0; k < c->N; ++k) {
                u64 &x = h[((size_t)p * nl + i) * c->N + k];
                if (x >= c->mod[i]) return fr_fail(FR_EINVAL, "import: residue not canonical (limb %d)", i);
            }
    FR_HIP(hipMemcpyAsync(dst, h.data(), w * 8, hipMemcpyHostToDevice, c->stream));
    frk::ntt_fwd(c, dst, nl, qmap(), npoly, (size_t)nl * c->N);
    FR_HIP(hipStreamSynchronize(c->stream));
    return FR_OK;
}

static int export_poly(fr_ctx *c, const u64 *src, int nl, int npoly, uint64_t *host) {
    c->arena.reset();
    Scope sc(c->arena);
    const size_t w = (size_t)npoly * nl * c->N;
    u64 *t = scratch(c, w);
    CHECK(t, FR_ENOMEM, "export: scratch");
    FR_HIP(hipMemcpyAsync(t, src, w * 8, hipMemcpyDeviceToDevice, c->stream));
    frk::ntt_inv(c, t, nl, qmap(), npoly, (size_t)nl * c->N);
    FR_HIP(hipMemcpyAsync(host, t, w * 8, hipMemcpyDeviceToHost, c->stream));
    FR_HIP(hipStreamSynchronize(c->stream));
    return FR_OK;
}

extern "C" int fr_pt_import(fr_ctx *c, const uint64_t *host, int32_t level, double scale, fr_pt *out) try {
    if (c) if (int e_ = no_capture(c, "fr_pt_import")) return e_;
    CHECK(c && host && out && out->data, FR_EINVAL, "fr_pt_import: null argument");
    CHECK(level >= 0 && level <= c->L && level <= out->cap, FR_EINVAL, "fr_pt_import: bad level");
    if (int e = import_poly(c, host, level + 1, 1, out->data)) return e;
    out->level = level;
    out->scale = scale;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_pt_export(fr_ctx *c, const fr_pt *p, uint64_t *host) try {
    if (c) if (int e_ = no_capture(c, "fr_pt_export")) return e_;
    CHECK(c && p && p->data && host, FR_EINVAL, "fr_pt_export: null argument");
    CHECK(p->level >= 0 && p->level <= c->L, FR_EINVAL, "fr_pt_export: bad level");
    return export_poly(c, p->data, p->level + 1, 1, host);
} FR_CATCH(c)

extern "C" int fr_ct_import(fr_ctx *c, const uint64_t *host, int32_t level, double scale, fr_ct *out) try {
    if (c) if (int e_ = no_capture(c, "fr_ct_import")) return e_;
    CHECK(c && host && out && out->data, FR_EINVAL, "fr_ct_import: null argument");
    CHECK(level >= 0 && level <= c->L && level <= out->cap, FR_EINVAL, "fr_ct_import: bad level");
    if (int e = import_poly(c, host, level + 1, 2, out->data)) return e;
    out->level = level;
    out->scale = scale;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_ct_export(fr_ctx *c, const fr_ct *x, uint64_t *host) try {
    if (c) if (int e_ = no_capture(c, "fr_ct_export")) return e_;
    CHECK(c && host, FR_EINVAL, "fr_ct_export: null argument");
    if (int e = check_ct(c, x, "fr_ct_export")) return e;
    return export_poly(c, x->data, x->level + 1, 2, host);
} FR_CATCH(c)

extern "C" int fr_encrypt(fr_ctx *c, const fr_keys *K, const fr_pt *p, uint64_t seed, fr_ct *out) try {
    if (int e = keys_ok(c, K, "fr_encrypt")) return e;
    CHECK(c && K && p && p->data, FR_EINVAL, "fr_encrypt: null argument");
    const int l = p->level;
    CHECK(l >= 0 && l <= c->L, FR_EINVAL, "fr_encrypt: bad plaintext level");
    if (int e = check_out(c, out, l, "fr_encrypt")) return e;
    c->arena.reset();
    Scope sc(c->arena);
    const int N = c->N;
    const size_t lw = (size_t)(l + 1) * N;
    u64 *v = scratch(c, 3 * lw);
    CHECK(v, FR_ENOMEM, "fr_encrypt: scratch");
    u64 *e0 = v + lw, *e1 = v + 2 * lw;
    frk::sample_small(c, v, seed, POLY_ENC_V, KIND_TERNARY, qmap(), l + 1);
    frk::sample_small(c, e0, seed, POLY_ENC_E0, KIND_GAUSS, qmap(), l + 1);
    frk::sample_small(c, e1, seed, POLY_ENC_E1, KIND_GAUSS, qmap(), l + 1);
    frk::ntt_fwd(c, v, l + 1, qmap(), 3, lw);
    frk::encrypt_combine(c, out->data, out->data + lw, v, e0, e1, p->data, K->pk, K->pk + (size_t)(c->L + 1) * N, l + 1);
    FR_HIP(hipGetLastError());
    out->level = l;
    out->scale = p->scale;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_decrypt(fr_ctx *c, const fr_keys *K, const fr_ct *x, fr_pt *out) try {
    if (int e = keys_ok(c, K, "fr_decrypt")) return e;
    CHECK(c && K && out && out->data, FR_EINVAL, "fr_decrypt: null argument");
    if (int e = check_ct(c, x, "fr_decrypt")) return e;
    CHECK(x->level <= out->cap, FR_EINVAL, "fr_decrypt: output capacity");
    const size_t lw = (size_t)(x->level + 1) * c->N;
    frk::decrypt_combine(c, out->data, x->data, x->data + lw, K->s_mont, x->level + 1);
    FR_HIP(hipGetLastError());
    out->level = x->level;
    out->scale = x->scale;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_decode(fr_ctx *c, const fr_pt *p, double *z, int32_t n) try {
    if (c) if (int e_ = no_capture(c, "fr_decode")) return e_;
    CHECK(c && p && p->data && z, FR_EINVAL, "fr_decode: null argument");
    CHECK(n >= 0 && n <= c->N / 2 && p->level >= 0 && p->level <= c->L, FR_EINVAL, "fr_decode: bad size or level");
    c->arena.reset();
    Scope sc(c->arena);
    const int N = c->N;
    const size_t lw = (size_t)(p->level + 1) * N;
    u64 *m = scratch(c, lw);
    double *work = (double *)c->arena.get((size_t)N * 16);
    double *zd = (double *)c->arena.get((size_t)N / 2 * 8);
    CHECK(m && work && zd, FR_ENOMEM, "fr_decode: scratch");
    FR_HIP(hipMemcpyAsync(m, p->data, lw * 8, hipMemcpyDeviceToDevice, c->stream));
    frk::ntt_inv(c, m, p->level + 1, qmap(), 1, 0);
    frk::decode_slots(c, zd, m, p->level, p->scale, work);
    if (n) FR_HIP(hipMemcpyAsync(z, zd, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    return flag_check(c, "fr_decode");
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// homomorphic operations
// ---------------------------------------------------------------------------
// scratch bytes one batched step may take before it is split into chunks
static const size_t kChunkBytes = (size_t)2 << 30;

static size_t arena_round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
// scratch of the hoisted rotations of nq inputs at `level`: before the
// rotation chunks (the staged c1 parts, the coefficient-form c1, the ModUp
// digits), and per rotation of a chunk (the key inner products U, the ModDown
// correction V, the P limbs of U in coefficient form)
static size_t rotation_base_bytes(const fr_ctx *c, int level, int nq) {
    const size_t N = c->N, lw = (size_t)(level + 1) * N, nE = level + 1 + c->nP;
    const size_t stage = nq > 1 ? arena_round((size_t)nq * lw * 8) : 0;
    return stage + arena_round((size_t)nq * lw * 8) + arena_round((size_t)nq * num_digits(c, level) * nE * N * 8);
}
static size_t rotation_scratch_bytes(const fr_ctx *c, int level, int nq) {
    const size_t N = c->N, lw = (size_t)(level + 1) * N, nE = level + 1 + c->nP;
    return (size_t)nq * (2 * nE * N + 2 * lw + 2 * c->nP * N) * 8;
}

// Hoisted rotations of nq ciphertexts (same level): outs[q * nrot + r] =
// Rot_{rots[r]}(in[q]).  ModUp of every c1 once, then per rotation the key
// inner product of all queries (one read of the key feeds every query), one
// batched ModDown preparation per chunk of rotations, and the fused finish.
static int rotate_hoisted_impl(fr_ctx *c, const fr_keys *K, const fr_ct *in, int nq, const int32_t *rots, int nrot,
                               fr_ct *outs, size_t chunk_bytes = kChunkBytes) {
    if (int e = keys_ok(c, K, "fr_rotate_hoisted")) return e;
    const int N = c->N, l = in[0].level, nE = l + 1 + c->nP;
    const size_t lw = (size_t)(l + 1) * N;
    for (int q = 0; q < nq; ++q) {
        if (int e = check_ct(c, &in[q], "fr_rotate_hoisted")) return e;
        CHECK(in[q].level == l, FR_ELEVEL, "fr_rotate_hoisted_batch: inputs differ in level");
    }
    std::vector<u64> gs(nrot);
    std::vector<int> live;  // rotations that need a key switch
    for (int r = 0; r < nrot; ++r) {
        gs[r] = galois_element(N, rots[r]);
        CHECK(gs[r] == 1 || K->find(gs[r]), FR_ENOKEY, "fr_rotate_hoisted: no key for rotation %d", rots[r]);
        if (gs[r] != 1) live.push_back(r);
    }
    for (int q = 0; q < nq; ++q)
        for (int r = 0; r < nrot; ++r) {
            fr_ct &o = outs[(size_t)q * nrot + r];
            if (int e = check_out(c, &o, l, "fr_rotate_hoisted")) return e;
            for (int q2 = 0; q2 < nq; ++q2)
                CHECK(o.data != in[q2].data, FR_EINVAL, "fr_rotate_hoisted: output aliases an input");
        }
    Scope sc(c->arena);
    const int nl = (int)live.size();
    if (nl) {
        const int ndig = num_digits(c, l);
        const size_t dstride = (size_t)ndig * nE * N;
        const u64 *c1 = in[0].data + lw;
        if (nq > 1) {  // stage the c1 parts contiguously for the batched ModUp
            u64 *C1 = scratch(c, (size_t)nq * lw);
            for (int q = 0; q < nq; ++q)
                FR_HIP(hipMemcpyAsync(C1 + (size_t)q * lw, in[q].data + lw, lw * 8, hipMemcpyDeviceToDevice,
                                      c->stream));
            c1 = C1;
        }
        u64 *D = scratch(c, (size_t)nq * dstride);
        ks_modup(c, c1, l, D, nq, lw);
        // per rotation of a chunk: U, V and the ModDown's P limbs
        const size_t per_rot = rotation_scratch_bytes(c, l, nq);
        const int rc = (int)std::max<size_t>(1, std::min<size_t>(nl, chunk_bytes / per_rot));
        std::vector<u64 *> op(nq);
        std::vector<const u64 *> ip(nq);
        for (int q = 0; q < nq; ++q) ip[q] = in[q].data;
        for (int r0 = 0; r0 < nl; r0 += rc) {
            Scope sc2(c->arena);
            const int rn = std::min(rc, nl - r0);
            const size_t ur = (size_t)nq * 2 * nE * N, vr = (size_t)nq * 2 * lw;
            u64 *U = scratch(c, rn * ur);
            u64 *V = scratch(c, rn * vr);
            for (int i = 0; i < rn; ++i) {
                const u64 g = gs[live[r0 + i]];
                u64 *Ui = U + i * ur;
                frk::ks_inner(c, Ui, Ui + (size_t)nE * N, D, K->find(g)->data, g, l, false, nq, dstride,
                              (size_t)2 * nE * N);
            }
            ks_moddown_prep(c, U, rn * nq, l, V);
            for (int i = 0; i < rn; ++i) {
                const int r = live[r0 + i];
                for (int q = 0; q < nq; ++q) op[q] = outs[(size_t)q * nrot + r].data;
                frk::moddown_rot(c, op.data(), U + i * ur, V + i * vr, ip.data(), gs[r], l, nq);
            }
        }
    }
    for (int q = 0; q < nq; ++q)
        for (int r = 0; r < nrot; ++r) {
            fr_ct &o = outs[(size_t)q * nrot + r];
            if (gs[r] == 1)
                FR_HIP(hipMemcpyAsync(o.data, in[q].data, 2 * lw * 8, hipMemcpyDeviceToDevice, c->stream));
            o.level = l;
            o.scale = in[q].scale;
        }
    FR_HIP(hipGetLastError());
    return FR_OK;
}

extern "C" int fr_rotate_hoisted(fr_ctx *c, const fr_keys *K, const fr_ct *in, const int32_t *rots, int32_t nrot,
                                 fr_ct *outs) try {
    CHECK(c && K && in && (nrot == 0 || (rots && outs)), FR_EINVAL, "fr_rotate_hoisted: null argument");
    c->arena.reset();
    return rotate_hoisted_impl(c, K, in, 1, rots, nrot, outs);
} FR_CATCH(c)

extern "C" int fr_rotate_hoisted_batch(fr_ctx *c, const fr_keys *K, const fr_ct *in, int32_t nq, const int32_t *rots,
                                       int32_t nrot, fr_ct *outs) try {
    CHECK(c && K && in && nq >= 1 && (nrot == 0 || (rots && outs)), FR_EINVAL,
          "fr_rotate_hoisted_batch: null argument or nq < 1");
    c->arena.reset();
    return rotate_hoisted_impl(c, K, in, nq, rots, nrot, outs);
} FR_CATCH(c)

// Allocation-free form of fr_rotate_hoisted: the same sequence with the
// context's arena swapped for the one-chunk arena over the fixed array (a
// vector swap: no allocation), rotations taken in chunks that fit beside the
// ModUp digits.  No kernel of the sequence reads scratch it has not written
// in the same call, so the array needs no clearing.
extern "C" int fr_rotate_hoisted_noalloc(fr_ctx *c, const fr_keys *K, const fr_ct *in, const int32_t *rots,
                                         int32_t nrot, fr_ct *outs) try {
    CHECK(c && K && in && (nrot == 0 || (rots && outs)), FR_EINVAL, "fr_rotate_hoisted_noalloc: null argument");
    if (int e = check_ct(c, in, "fr_rotate_hoisted_noalloc")) return e;
    CHECK(!c->fixed_arena.chunks.empty(), FR_EHIP, "fr_rotate_hoisted_noalloc: no fixed scratch on this device");
    const size_t base = rotation_base_bytes(c, in->level, 1), per = rotation_scratch_bytes(c, in->level, 1);
    CHECK(base + per <= FR_NOALLOC_SCRATCH_BYTES, FR_ENOMEM,
          "fr_rotate_hoisted_noalloc: a rotation at level %d needs %zu bytes of scratch, the fixed array holds %zu",
          in->level, base + per, (size_t)FR_NOALLOC_SCRATCH_BYTES);
    struct Swap {
        fr_ctx *c;
        explicit Swap(fr_ctx *cc) : c(cc) {
            c->fixed_arena.chunks[0].used = 0;
            c->fixed_arena.hold = 0;
            std::swap(c->arena, c->fixed_arena);
        }
        ~Swap() { std::swap(c->arena, c->fixed_arena); }
    } swap(c);
    return rotate_hoisted_impl(c, K, in, 1, rots, nrot, outs, FR_NOALLOC_SCRATCH_BYTES - base);
} FR_CATCH(c)

extern "C" int fr_rescale(fr_ctx *c, const fr_ct *in, fr_ct *out) try {
    CHECK(c, FR_EINVAL, "null context");
    if (int e = check_ct(c, in, "fr_rescale")) return e;
    CHECK(in->level >= 1, FR_ELEVEL, "fr_rescale: level 0 cannot be rescaled");
    if (int e = check_out(c, out, in->level - 1, "fr_rescale")) return e;
    CHECK(out->data != in->data, FR_EINVAL, "fr_rescale: output aliases input");
    c->arena.reset();
    rescale_dev(c, in->data, in->level, out->data);
    FR_HIP(hipGetLastError());
    out->scale = in->scale / (double)c->mod[in->level];
    out->level = in->level - 1;
    return FR_OK;
} FR_CATCH(c)

static int addsub(fr_ctx *c, const fr_ct *a, const fr_ct *b, fr_ct *out, bool sub) {
    CHECK(c, FR_EINVAL, "null context");
    if (int e = check_ct(c, a, "fr_add")) return e;
    if (int e = check_ct(c, b, "fr_add")) return e;
    CHECK(a->level == b->level, FR_ELEVEL, "fr_add: level mismatch %d vs %d", a->level, b->level);
    if (int e = check_out(c, out, a->level, "fr_add")) return e;
    const size_t lw = (size_t)(a->level + 1) * c->N;
    frk::add(c, out->data, a->data, b->data, a->level + 1, 2, lw, lw, lw, sub);
    FR_HIP(hipGetLastError());
    out->level = a->level;
    out->scale = a->scale;
    return FR_OK;
}
extern "C" int fr_add(fr_ctx *c, const fr_ct *a, const fr_ct *b, fr_ct *out) { return addsub(c, a, b, out, false); }
extern "C" int fr_sub(fr_ctx *c, const fr_ct *a, const fr_ct *b, fr_ct *out) { return addsub(c, a, b, out, true); }

// Encrypted-database product: Rescale(Relin(sum_k a[k] (x) b[k])), the
// degree-2 sum relinearised once.
extern "C" int fr_tensor_sum_relin_rescale(fr_ctx *c, const fr_keys *K, const fr_ct *a, const fr_ct *b, int32_t n,
                                           fr_ct *out) try {
    if (int e = keys_ok(c, K, "fr_tensor_sum_relin_rescale")) return e;
    CHECK(c && K && a && b && out && n >= 1, FR_EINVAL, "fr_tensor_sum_relin_rescale: null argument or no pair");
    const int l = a[0].level;
    for (int k = 0; k < n; ++k) {
        if (int e = check_ct(c, &a[k], "fr_tensor_sum_relin_rescale")) return e;
        if (int e = check_ct(c, &b[k], "fr_tensor_sum_relin_rescale")) return e;
        CHECK(a[k].level == l && b[k].level == l, FR_ELEVEL, "fr_tensor_sum_relin_rescale: level mismatch");
        CHECK(a[k].scale * b[k].scale == a[0].scale * b[0].scale, FR_ELEVEL,
              "fr_tensor_sum_relin_rescale: the products differ in scale");
    }
    CHECK(l >= 1, FR_ELEVEL, "fr_tensor_sum_relin_rescale: no level left");
    if (int e = check_out(c, out, l - 1, "fr_tensor_sum_relin_rescale")) return e;
    const KeyEntry *rk = K->find(0);
    CHECK(rk, FR_ENOKEY, "fr_tensor_sum_relin_rescale: relinearisation key missing");
    c->arena.reset();
    Scope sc(c->arena);
    const int N = c->N, nE = l + 1 + c->nP;
    const size_t lw = (size_t)(l + 1) * N;
    std::vector<const u64 *> pa(n), pb(n);
    for (int k = 0; k < n; ++k) {
        pa[k] = a[k].data;
        pb[k] = b[k].data;
    }
    u64 *T01 = scratch(c, 2 * lw), *T2 = scratch(c, lw);
    frk::tensor_sum(c, T01, T2, l + 1, n, pa.data(), pb.data());
    u64 *D = scratch(c, (size_t)num_digits(c, l) * nE * N);
    ks_modup(c, T2, l, D);
    u64 *U = scratch(c, (size_t)2 * nE * N);
    frk::ks_inner(c, U, U + (size_t)nE * N, D, rk->data, 1, l, false, 1, 0, 0, relin_folds(c) ? T01 : nullptr, 0);
    relin_rescale_into(c, T01, U, 1, l, out->data);
    FR_HIP(hipGetLastError());
    out->level = l - 1;
    out->scale = (a[0].scale * b[0].scale) / (double)c->mod[l];
    return FR_OK;
} FR_CATCH(c)

// Membership aggregation: the group ciphertexts are added, then every slot
// receives the sum of all N/2 slots through log2(N/2) doublings
// x <- x + Rot_{2^i}(x), each one key switch.
extern "C" int fr_membership_aggregate(fr_ctx *c, const fr_keys *K, const fr_ct *in, int32_t n, fr_ct *out) try {
    if (int e = keys_ok(c, K, "fr_membership_aggregate")) return e;
    CHECK(c && K && in && out && n >= 1, FR_EINVAL, "fr_membership_aggregate: null argument or no input");
    const int l = in[0].level;
    for (int i = 0; i < n; ++i) {
        if (int e = check_ct(c, &in[i], "fr_membership_aggregate")) return e;
        CHECK(in[i].level == l && in[i].scale == in[0].scale, FR_ELEVEL,
              "fr_membership_aggregate: inputs differ in level or scale");
        CHECK(in[i].data != out->data, FR_EINVAL, "fr_membership_aggregate: output aliases an input");
    }
    if (int e = check_out(c, out, l, "fr_membership_aggregate")) return e;
    const int slots_log = c->logN - 1;
    for (int i = 0; i < slots_log; ++i)
        CHECK(K->find(galois_element(c->N, 1 << i)), FR_ENOKEY, "fr_membership_aggregate: no key for rotation %d",
              1 << i);
    c->arena.reset();
    Scope sc(c->arena);
    const size_t lw = (size_t)(l + 1) * c->N;
    if (n == 1)
        FR_HIP(hipMemcpyAsync(out->data, in[0].data, 2 * lw * 8, hipMemcpyDeviceToDevice, c->stream));
    else
        frk::add(c, out->data, in[0].data, in[1].data, l + 1, 2, lw, lw, lw, false);
    for (int i = 2; i < n; ++i) frk::add(c, out->data, out->data, in[i].data, l + 1, 2, lw, lw, lw, false);
    out->level = l;
    out->scale = in[0].scale;
    fr_ct tmp{scratch(c, 2 * lw), l, l, 0.0};
    for (int i = 0; i < slots_log; ++i) {
        const int32_t r = 1 << i;
        if (int e = rotate_hoisted_impl(c, K, out, 1, &r, 1, &tmp)) return e;
        frk::add(c, out->data, out->data, tmp.data, l + 1, 2, lw, lw, lw, false);
    }
    FR_HIP(hipGetLastError());
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_mul_plain(fr_ctx *c, const fr_ct *a, const fr_pt *p, fr_ct *out) try {
    CHECK(c && p && p->data, FR_EINVAL, "fr_mul_plain: null argument");
    if (int e = check_ct(c, a, "fr_mul_plain")) return e;
    const int l = std::min(a->level, p->level);
    if (int e = check_out(c, out, l, "fr_mul_plain")) return e;
    const size_t la = (size_t)(a->level + 1) * c->N, lo = (size_t)(l + 1) * c->N;
    CHECK(out->data != a->data || l == a->level, FR_EINVAL, "fr_mul_plain: aliasing with a level change");
    frk::mul_pt(c, out->data, a->data, p->data, l + 1, 2, lo, la);
    FR_HIP(hipGetLastError());
    out->level = l;
    out->scale = a->scale * p->scale;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_mul_relin_rescale(fr_ctx *c, const fr_keys *K, const fr_ct *a, const fr_ct *b, fr_ct *out) try {
    if (int e = keys_ok(c, K, "fr_mul_relin_rescale")) return e;
    CHECK(c && K, FR_EINVAL, "null argument");
    if (int e = check_ct(c, a, "fr_mul_relin_rescale")) return e;
    if (int e = check_ct(c, b, "fr_mul_relin_rescale")) return e;
    CHECK(a->level == b->level, FR_ELEVEL, "fr_mul_relin_rescale: level mismatch");
    CHECK(a->level >= 1, FR_ELEVEL, "fr_mul_relin_rescale: no level left");
    if (int e = check_out(c, out, a->level - 1, "fr_mul_relin_rescale")) return e;
    c->arena.reset();
    Ct A{a->data, a->level, a->scale}, B{b->data, b->level, b->scale};
    if (int e = mul_relin_rescale_dev(c, K, A, B, out->data)) return e;
    FR_HIP(hipGetLastError());
    out->level = a->level - 1;
    out->scale = (a->scale * b->scale) / (double)c->mod[a->level];
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_mul_int(fr_ctx *c, const fr_ct *a, int64_t k, fr_ct *out) try {
    CHECK(c, FR_EINVAL, "null context");
    if (int e = check_ct(c, a, "fr_mul_int")) return e;
    if (int e = check_out(c, out, a->level, "fr_mul_int")) return e;
    const size_t lw = (size_t)(a->level + 1) * c->N;
    mul_int_dev(c, a->data, lw, a->level + 1, (long long)k, out->data, lw);
    FR_HIP(hipGetLastError());
    out->level = a->level;
    out->scale = a->scale * (double)k;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_add_const(fr_ctx *c, const fr_ct *a, double cst, fr_ct *out) try {
    CHECK(c, FR_EINVAL, "null context");
    if (int e = check_ct(c, a, "fr_add_const")) return e;
    if (int e = check_out(c, out, a->level, "fr_add_const")) return e;
    const size_t lw = (size_t)(a->level + 1) * c->N;
    if (out->data != a->data) FR_HIP(hipMemcpyAsync(out->data, a->data, 2 * lw * 8, hipMemcpyDeviceToDevice, c->stream));
    add_const_dev(c, out->data, a->level, cst, a->scale);
    FR_HIP(hipGetLastError());
    out->level = a->level;
    out->scale = a->scale;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_drop_to(fr_ctx *c, const fr_ct *a, int32_t level, fr_ct *out) try {
    CHECK(c, FR_EINVAL, "null context");
    if (int e = check_ct(c, a, "fr_drop_to")) return e;
    CHECK(level >= 0 && level <= a->level, FR_ELEVEL, "fr_drop_to: bad level");
    if (int e = check_out(c, out, level, "fr_drop_to")) return e;
    CHECK(out->data != a->data || level == a->level, FR_EINVAL, "fr_drop_to: aliasing");
    const size_t lw = (size_t)(level + 1) * c->N;
    for (int p = 0; p < 2; ++p)
        FR_HIP(hipMemcpyAsync(out->data + p * lw, a->data + (size_t)p * (a->level + 1) * c->N, lw * 8,
                              hipMemcpyDeviceToDevice, c->stream));
    out->level = level;
    out->scale = a->scale;
    return FR_OK;
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// database
// ---------------------------------------------------------------------------
extern "C" void fr_db_destroy(fr_db *db) {
    if (!db) return;
    (void)hipStreamSynchronize(db->ctx->stream);
    (void)hipFree(db->data);
    delete db;
}

extern "C" int fr_db_groups(const fr_db *db) { return db ? db->G : 0; }

// byte layout of a diagonal of nl limbs at level `level` (limbs past the
// level are the special primes): limbs of moduli below 2^40 packed in 5 B
static size_t db_layout(const fr_ctx *c, int level, int nl, DbLayout &lay) {
    size_t o = 0;
    for (int m = 0; m < nl; ++m) {
        const u64 q = c->mod[m <= level ? m : c->L + 1 + (m - level - 1)];
        lay.packed[m] = q < (1ull << 40);
        lay.off[m] = (unsigned)o;
        o += (lay.packed[m] ? 5 : 8) * (size_t)c->N;
    }
    return o;
}

static int db_alloc(fr_ctx *c, int G, int ell, int B, int n1, int level, double scale, fr_db **out) {
    CHECK(level + 1 + c->nP <= kDbMaxLimbs, FR_EINVAL, "fr_db: at most %d limbs per diagonal", kDbMaxLimbs);
    fr_db *db = new fr_db();
    db->ctx = c;
    db->G = G;
    db->ell = ell;
    db->B = B;
    db->n1 = n1;
    db->level = level;
    db->nl = level + 1;
    db->scale = scale;
    db->stride = db_layout(c, level, db->nl, db->lay);
    if (hipMalloc(&db->data, (size_t)G * ell * db->stride) != hipSuccess) {
        delete db;
        return fr_fail(FR_ENOMEM, "fr_db: cannot allocate %zu bytes of diagonals", (size_t)G * ell * db->stride);
    }
    *out = db;
    return FR_OK;
}

extern "C" int fr_db_load(fr_ctx *c, const float *T, int32_t K, int32_t ell, int32_t B, int32_t n1, int32_t level,
                          double scale, fr_db **out) try {
    if (c) if (int e_ = no_capture(c, "fr_db_load")) return e_;
    CHECK(c && out && (K == 0 || T), FR_EINVAL, "fr_db_load: null argument");
    const int h = c->N / 2;
    CHECK(K >= 0 && ell > 0 && B > 0 && (long long)B * ell <= h && n1 > 0 && n1 <= ell && level >= 0 &&
              level <= c->L,
          FR_EINVAL, "fr_db_load: bad layout");
    const int G = std::max(1, (int)((K + (long long)B * ell - 1) / ((long long)B * ell)));
    fr_db *db = nullptr;
    if (int e = db_alloc(c, G, ell, B, n1, level, scale, &db)) return e;
    std::unique_ptr<fr_db, void (*)(fr_db *)> guard(db, fr_db_destroy);
    c->arena.reset();
    Scope sc(c->arena);
    float *Td = (float *)c->arena.get((size_t)std::max(K, 1) * ell * 4);
    CHECK(Td, FR_ENOMEM, "fr_db_load: scratch");
    if (K) FR_HIP(hipMemcpyAsync(Td, T, (size_t)K * ell * 4, hipMemcpyHostToDevice, c->stream));
    FR_HIP(hipStreamSynchronize(c->stream));
    const int batch = std::min(ell, 32);
    double *slots = (double *)c->arena.get((size_t)batch * h * 8);
    double *work = (double *)c->arena.get((size_t)batch * c->N * 16);
    CHECK(slots && work, FR_ENOMEM, "fr_db_load: scratch");
    const size_t pw = (size_t)(level + 1) * c->N;
    u64 *dst = scratch(c, (size_t)batch * pw);
    for (int g = 0; g < G; ++g)
        for (int d0 = 0; d0 < ell; d0 += batch) {
            const int nd = std::min(batch, ell - d0);
            frk::db_slots(c, slots, Td, K, ell, B, n1, g, d0, nd);
            frk::encode_slots(c, dst, slots, h, level, scale, nd, (size_t)h, pw, work);
            frk::ntt_fwd(c, dst, level + 1, qmap(), nd, pw);
            frk::mont_scale(c, dst, level + 1, qmap(), nd, pw, true);
            frk::db_pack(c, db->data + ((size_t)g * ell + d0) * db->stride, db->stride, db->lay, dst, level + 1, nd);
        }
    if (int e = flag_check(c, "fr_db_load")) return e;
    *out = guard.release();
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_db_import(fr_ctx *c, const uint64_t *host, int32_t G, int32_t ell, int32_t B, int32_t n1,
                            int32_t level, double scale, fr_db **out) try {
    if (c) if (int e_ = no_capture(c, "fr_db_import")) return e_;
    CHECK(c && host && out, FR_EINVAL, "fr_db_import: null argument");
    CHECK(G >= 1 && ell > 0 && B > 0 && (long long)B * ell <= c->N / 2 && n1 > 0 && n1 <= ell && level >= 0 &&
              level <= c->L,
          FR_EINVAL, "fr_db_import: bad layout");
    fr_db *db = nullptr;
    if (int e = db_alloc(c, G, ell, B, n1, level, scale, &db)) return e;
    std::unique_ptr<fr_db, void (*)(fr_db *)> guard(db, fr_db_destroy);
    const size_t pw = (size_t)(level + 1) * c->N;
    c->arena.reset();
    Scope sc(c->arena);
    const int batch = 32;
    u64 *t = scratch(c, (size_t)batch * pw);
    for (int p0 = 0; p0 < G * ell; p0 += batch) {
        const int nd = std::min(batch, G * ell - p0);
        for (int p = 0; p < nd; ++p)
            if (int e = import_poly(c, host + (size_t)(p0 + p) * pw, level + 1, 1, t + p * pw)) return e;
        frk::mont_scale(c, t, level + 1, qmap(), nd, pw, true);
        frk::db_pack(c, db->data + (size_t)p0 * db->stride, db->stride, db->lay, t, level + 1, nd);
    }
    FR_HIP(hipStreamSynchronize(c->stream));
    *out = guard.release();
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_db_export(fr_ctx *c, const fr_db *db, int32_t g, int32_t d, uint64_t *host) try {
    if (int e = db_ok(c, db, "fr_db_export")) return e;
    if (c) if (int e_ = no_capture(c, "fr_db_export")) return e_;
    CHECK(c && db && host, FR_EINVAL, "fr_db_export: null argument");
    CHECK(g >= 0 && g < db->G && d >= 0 && d < db->ell, FR_EINVAL, "fr_db_export: bad index");
    c->arena.reset();
    Scope sc(c->arena);
    const size_t pw = (size_t)(db->level + 1) * c->N;
    u64 *t = scratch(c, pw);
    CHECK(t, FR_ENOMEM, "fr_db_export: scratch");
    frk::db_unpack(c, t, db->data + ((size_t)g * db->ell + d) * db->stride, db->stride, db->lay, db->level + 1, 1);
    frk::mont_scale(c, t, db->level + 1, qmap(), 1, 0, false);
    frk::ntt_inv(c, t, db->level + 1, qmap(), 1, 0);
    FR_HIP(hipMemcpyAsync(host, t, pw * 8, hipMemcpyDeviceToHost, c->stream));
    FR_HIP(hipStreamSynchronize(c->stream));
    return FR_OK;
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// the BSGS diagonal matrix-vector product
// ---------------------------------------------------------------------------
// BSGS-Diagonal products of nq queries, query q against group groups[q] of
// dbs[q] (every database with the same ell, n1 and level): baby[q * n1 + i]
// is baby step i of query q, out[q] its score ciphertext.  Queries are
// ordered by diagonal group and run in chunks of up to the matvec chunk knob: one
// read of every diagonal per chunk and group (the MAC), the n2 rescales of
// every query in one batch, one ModUp batch of all giant-step inputs, per
// giant step one key read for the whole chunk, and one ModDown per query.

// Giant steps of qn queries from their rescaled inner sums R =
// [qn][n2][2][l+1][N]: out[q] = R_{q,0} + sum_j Rot_{j n1}(R_{q,j}), every
// rotation's key inner product summed over Q_l U P before one ModDown per
// query (Eq. bsgs2).
// c0_summed: R_{q,0}.c0 already holds the first polynomials' rotated sum
// (the R_{q,j}.c0 of j >= 1 are not read)
static int giant_steps(fr_ctx *c, const fr_keys *K, const u64 *R, int qn, int n2, int n1, int l, u64 *const *outp,
                       bool c0_summed = false) {
    Scope sc(c->arena);
    const int N = c->N, nE = l + 1 + c->nP, ndig = num_digits(c, l);
    const size_t rw = (size_t)2 * (l + 1) * N, lwl = (size_t)(l + 1) * N, dstride = (size_t)ndig * nE * N;
    // S_q = R_{q,0} + sum_j sigma_j(R_{q,j}.c0) + ModDown(sum_j KS_j); staged
    // contiguously unless there is a single query
    u64 *S = qn == 1 ? outp[0] : scratch(c, (size_t)qn * rw);
    CHECK(S, FR_ENOMEM, "giant steps: scratch");
    if (qn == 1)
        FR_HIP(hipMemcpyAsync(S, R, rw * 8, hipMemcpyDeviceToDevice, c->stream));
    else
        FR_HIP(hipMemcpy2DAsync(S, rw * 8, R, n2 * rw * 8, rw * 8, qn, hipMemcpyDeviceToDevice, c->stream));
    if (n2 > 1) {
        // ModUp of every R_{q,j}.c1 (flat item f = q n2 + j, f >= 1; the
        // j = 0 items of later queries are converted and left unused)
        u64 *D = scratch(c, ((size_t)qn * n2 - 1) * dstride);
        u64 *U = scratch(c, (size_t)qn * 2 * nE * N);
        CHECK(D && U, FR_ENOMEM, "giant steps: scratch");
        ks_modup(c, R + rw + lwl, l, D, qn * n2 - 1, rw);
        std::vector<const unsigned char *> kp(n2 - 1);
        std::vector<u64> gp(n2 - 1);
        for (int j = 1; j < n2; ++j) {
            gp[j - 1] = galois_element(N, j * n1);
            kp[j - 1] = K->find(gp[j - 1])->data;
        }
        // all giant-step key inner products summed in one pass per chunk
        const int chunk = frk::ks_inner_sum_chunk(c, l);
        for (int j0 = 0; j0 < n2 - 1; j0 += chunk) {
            const int nj = std::min(chunk, n2 - 1 - j0);
            frk::ks_inner_sum(c, U, U + (size_t)nE * N, D + (size_t)j0 * dstride, kp.data() + j0, gp.data() + j0, nj,
                              dstride, l, j0 > 0, qn, (size_t)n2 * dstride, (size_t)2 * nE * N);
        }
        if (!c0_summed) frk::automorph_sum(c, S, R + rw, gp.data(), n2 - 1, l + 1, qn, rw, rw, (size_t)n2 * rw);
        ks_moddown_into(c, U, qn, l, S, lwl, true);
    }
    if (qn > 1)
        for (int qq = 0; qq < qn; ++qq)
            FR_HIP(hipMemcpyAsync(outp[qq], S + (size_t)qq * rw, rw * 8, hipMemcpyDeviceToDevice, c->stream));
    return FR_OK;
}

static int matvec_impl(fr_ctx *c, const fr_keys *K, const fr_ct *baby, int nq, int n1, const fr_db *const *dbs,
                       const int32_t *groups, fr_ct *out) {
    if (int e = keys_ok(c, K, "fr_bsgs_diag_matvec")) return e;
    const fr_db *db0 = dbs[0];
    for (int q = 0; q < nq; ++q) {
        const fr_db *db = dbs[q];
        if (int e = db_ok(c, db, "fr_bsgs_diag_matvec")) return e;
        CHECK(n1 == db->n1, FR_EINVAL, "fr_bsgs_diag_matvec: n1 %d differs from the database's %d", n1, db->n1);
        CHECK(groups[q] >= 0 && groups[q] < db->G, FR_EINVAL, "fr_bsgs_diag_matvec: group %d out of range",
              groups[q]);
        CHECK(db->ell == db0->ell && db->level == db0->level && db->nl == db0->nl, FR_EINVAL,
              "fr_bsgs_diag_matvec_batch: databases differ in ell, level or extension");
    }
    const int N = c->N, ell = db0->ell, bl = baby[0].level;
    for (int t = 0; t < nq * n1; ++t) {
        if (int e = check_ct(c, &baby[t], "fr_bsgs_diag_matvec")) return e;
        CHECK(baby[t].level == bl && baby[t].scale == baby[(t / n1) * n1].scale, FR_ELEVEL,
              "fr_bsgs_diag_matvec: baby steps differ in level or scale");
    }
    const int lv = std::min(bl, db0->level);
    CHECK(lv >= 1, FR_ELEVEL, "fr_bsgs_diag_matvec: no level left to rescale");
    const int n2 = (ell + n1 - 1) / n1, l = lv - 1;
    for (int j = 1; j < n2; ++j)
        CHECK(K->find(galois_element(N, j * n1)), FR_ENOKEY, "fr_bsgs_diag_matvec: no key for giant step %d", j * n1);
    for (int q = 0; q < nq; ++q) {
        if (int e = check_out(c, &out[q], l, "fr_bsgs_diag_matvec")) return e;
        for (int t = 0; t < nq * n1; ++t)
            CHECK(out[q].data != baby[t].data, FR_EINVAL, "fr_bsgs_diag_matvec: output aliases a baby step");
    }
    const size_t pw = (size_t)2 * (lv + 1) * N, rw = (size_t)2 * (l + 1) * N;
    auto diag_of = [&](int q) { return (const unsigned char *)(dbs[q]->data + (size_t)groups[q] * ell * dbs[q]->stride); };
    std::vector<int> order(nq);
    for (int q = 0; q < nq; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return diag_of(a) < diag_of(b); });
    const int chunk = c->tune[FR_TUNE_MATVEC_CHUNK];
    for (int q0 = 0; q0 < nq; q0 += chunk) {
        Scope sc(c->arena);
        const int qn = std::min(chunk, nq - q0);
        u64 *P = scratch(c, (size_t)qn * n2 * pw);
        u64 *R = scratch(c, (size_t)qn * n2 * rw);
        std::vector<const u64 *> bp((size_t)qn * n1);
        std::vector<const unsigned char *> dp(qn);
        for (int qq = 0; qq < qn; ++qq) {
            const int q = order[q0 + qq];
            dp[qq] = diag_of(q);
            for (int i = 0; i < n1; ++i) bp[(size_t)qq * n1 + i] = baby[(size_t)q * n1 + i].data;
        }
        frk::bsgs_mac(c, P, (size_t)n2 * pw, bp.data(), qn, n1, dp.data(), db0->stride, db0->lay, ell, lv, bl);
        rescale_dev(c, P, lv, R, qn * n2);
        std::vector<u64 *> op(qn);
        for (int qq = 0; qq < qn; ++qq) op[qq] = out[order[q0 + qq]].data;
        if (int e = giant_steps(c, K, R, qn, n2, n1, l, op.data())) return e;
    }
    FR_HIP(hipGetLastError());
    for (int q = 0; q < nq; ++q) {
        out[q].level = l;
        out[q].scale = (baby[(size_t)q * n1].scale * dbs[q]->scale) / (double)c->mod[lv];
    }
    return FR_OK;
}

extern "C" int fr_bsgs_diag_matvec(fr_ctx *c, const fr_keys *K, const fr_ct *baby, int32_t n1, const fr_db *db,
                                   int32_t group, fr_ct *out) try {
    CHECK(c && K && baby && db && out && n1 >= 1, FR_EINVAL, "fr_bsgs_diag_matvec: null argument");
    c->arena.reset();
    return matvec_impl(c, K, baby, 1, n1, &db, &group, out);
} FR_CATCH(c)

extern "C" int fr_bsgs_diag_matvec_batch(fr_ctx *c, const fr_keys *K, const fr_ct *baby, int32_t nq, int32_t n1,
                                         const fr_db *const *dbs, const int32_t *groups, fr_ct *out) try {
    CHECK(c && K && baby && dbs && groups && out && n1 >= 1 && nq >= 1, FR_EINVAL,
          "fr_bsgs_diag_matvec_batch: null argument or empty batch");
    c->arena.reset();
    return matvec_impl(c, K, baby, nq, n1, dbs, groups, out);
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// giant-step rotate-sum and the encrypted-database BSGS product
// ---------------------------------------------------------------------------
// checks shared by the two: n inputs of one level and scale, keys for the
// rotations j * stride (1 <= j < n), the output's capacity and aliasing
static int rotate_sum_checks(fr_ctx *c, const fr_keys *K, const fr_ct *in, int n, int stride, const fr_ct *out,
                             int out_level, const char *what) {
    for (int j = 0; j < n; ++j) {
        if (int e = check_ct(c, &in[j], what)) return e;
        CHECK(in[j].level == in[0].level && in[j].scale == in[0].scale, FR_ELEVEL, "%s: inputs differ in level or scale",
              what);
        CHECK(in[j].data != out->data, FR_EINVAL, "%s: output aliases an input", what);
    }
    for (int j = 1; j < n; ++j)
        CHECK(K->find(galois_element(c->N, j * stride)), FR_ENOKEY, "%s: no key for rotation %d", what, j * stride);
    return check_out(c, out, out_level, what);
}

extern "C" int fr_rotate_sum(fr_ctx *c, const fr_keys *K, const fr_ct *in, int32_t n, int32_t stride,
                             fr_ct *out) try {
    CHECK(c && K && in && out && n >= 1, FR_EINVAL, "fr_rotate_sum: null argument or no input");
    if (int e = keys_ok(c, K, "fr_rotate_sum")) return e;
    const int l = in[0].level;
    if (int e = rotate_sum_checks(c, K, in, n, stride, out, l, "fr_rotate_sum")) return e;
    c->arena.reset();
    Scope sc(c->arena);
    const size_t rw = (size_t)2 * (l + 1) * c->N;
    u64 *R = scratch(c, (size_t)n * rw);  // the inputs staged contiguously
    for (int j = 0; j < n; ++j)
        FR_HIP(hipMemcpyAsync(R + j * rw, in[j].data, rw * 8, hipMemcpyDeviceToDevice, c->stream));
    u64 *op = out->data;
    if (int e = giant_steps(c, K, R, 1, n, stride, l, &op)) return e;
    FR_HIP(hipGetLastError());
    out->level = l;
    out->scale = in[0].scale;
    return FR_OK;
} FR_CATCH(c)

// P_j = Rescale(Relin(sum_i baby[i] (x) diag[j n1 + i])) for every giant step
// j (the tensor sums, one ModUp batch, one read of the relinearisation key
// and one merged ModDown + rescale for all of them), then
// out = P_0 + sum_{j >= 1} Rot_{j n1}(P_j) with one shared ModDown.
extern "C" int fr_bsgs_encrypted_matvec(fr_ctx *c, const fr_keys *K, const fr_ct *baby, int32_t n1, const fr_ct *diag,
                                        int32_t ell, fr_ct *out) try {
    CHECK(c && K && baby && diag && out && n1 >= 1 && ell >= 1 && n1 <= ell, FR_EINVAL,
          "fr_bsgs_encrypted_matvec: null argument or bad shape");
    if (int e = keys_ok(c, K, "fr_bsgs_encrypted_matvec")) return e;
    const int l = baby[0].level, N = c->N, n2 = (ell + n1 - 1) / n1;
    for (int i = 0; i < n1; ++i) {
        if (int e = check_ct(c, &baby[i], "fr_bsgs_encrypted_matvec")) return e;
        CHECK(baby[i].level == l && baby[i].scale == baby[0].scale, FR_ELEVEL,
              "fr_bsgs_encrypted_matvec: baby steps differ in level or scale");
    }
    for (int d = 0; d < ell; ++d) {
        if (int e = check_ct(c, &diag[d], "fr_bsgs_encrypted_matvec")) return e;
        CHECK(diag[d].level == l && diag[d].scale == diag[0].scale, FR_ELEVEL,
              "fr_bsgs_encrypted_matvec: diagonals differ from the baby steps in level or scale");
        CHECK(diag[d].data != out->data, FR_EINVAL, "fr_bsgs_encrypted_matvec: output aliases a diagonal");
    }
    for (int i = 0; i < n1; ++i)
        CHECK(baby[i].data != out->data, FR_EINVAL, "fr_bsgs_encrypted_matvec: output aliases a baby step");
    CHECK(l >= 1, FR_ELEVEL, "fr_bsgs_encrypted_matvec: no level left to rescale");
    const KeyEntry *rk = K->find(0);
    CHECK(rk, FR_ENOKEY, "fr_bsgs_encrypted_matvec: relinearisation key missing");
    for (int j = 1; j < n2; ++j)
        CHECK(K->find(galois_element(N, j * n1)), FR_ENOKEY, "fr_bsgs_encrypted_matvec: no key for giant step %d",
              j * n1);
    if (int e = check_out(c, out, l - 1, "fr_bsgs_encrypted_matvec")) return e;
    c->arena.reset();
    Scope sc(c->arena);
    const int nE = l + 1 + c->nP, ndig = num_digits(c, l);
    const size_t lw = (size_t)(l + 1) * N, cw = 2 * lw, dstride = (size_t)ndig * nE * N;
    u64 *T01 = scratch(c, (size_t)n2 * cw), *T2 = scratch(c, (size_t)n2 * lw);
    std::vector<const u64 *> pa(n1), pb(n1);
    for (int j = 0; j < n2; ++j) {
        const int nj = std::min(n1, ell - j * n1);
        for (int i = 0; i < nj; ++i) {
            pa[i] = baby[i].data;
            pb[i] = diag[j * n1 + i].data;
        }
        frk::tensor_sum(c, T01 + j * cw, T2 + j * lw, l + 1, nj, pa.data(), pb.data());
    }
    u64 *D = scratch(c, (size_t)n2 * dstride);
    ks_modup(c, T2, l, D, n2, lw);
    u64 *U = scratch(c, (size_t)n2 * 2 * nE * N);
    frk::ks_inner(c, U, U + (size_t)nE * N, D, rk->data, 1, l, false, n2, dstride, (size_t)2 * nE * N,
                  relin_folds(c) ? T01 : nullptr, cw);
    u64 *R = scratch(c, (size_t)n2 * 2 * l * N);
    relin_rescale_into(c, T01, U, n2, l, R);
    u64 *op = out->data;
    if (int e = giant_steps(c, K, R, 1, n2, n1, l - 1, &op)) return e;
    FR_HIP(hipGetLastError());
    out->level = l - 1;
    out->scale = (baby[0].scale * diag[0].scale) / (double)c->mod[l];
    return FR_OK;
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// the BSGS product with the baby steps' ModDown hoisted past the inner sums
// ---------------------------------------------------------------------------
// Appends to every diagonal its residues mod the special primes, those of
// the plaintext's centered integer coefficients (exact mixed-radix lift).
extern "C" int fr_db_extend(fr_ctx *c, fr_db *db) try {
    if (c) if (int e_ = no_capture(c, "fr_db_extend")) return e_;
    CHECK(c && db, FR_EINVAL, "fr_db_extend: null argument");
    CHECK(db->ctx == c, FR_EINVAL, "fr_db_extend: database of another context");
    const int N = c->N, l = db->level, L1 = l + 1, nP = c->nP, nE = L1 + nP;
    if (db->nl == nE) return FR_OK;
    DbLayout lay{};
    const size_t stride = db_layout(c, l, nE, lay);
    const size_t nd = (size_t)db->G * db->ell, lw = (size_t)L1 * N, ew = (size_t)nE * N, pw = (size_t)nP * N;
    unsigned char *ext = nullptr;
    if (hipMalloc(&ext, nd * stride) != hipSuccess) {
        (void)hipGetLastError();
        return fr_fail(FR_ENOMEM, "fr_db_extend: cannot allocate %zu bytes of diagonals", nd * stride);
    }
    struct ExtGuard {  // frees the new buffer unless it replaces the old one
        unsigned char *&p;
        fr_ctx *c;
        ~ExtGuard() {
            if (p) {
                (void)hipStreamSynchronize(c->stream);
                (void)hipFree(p);
            }
        }
    } ext_guard{ext, c};
    c->arena.reset();
    Scope sc(c->arena);
    const size_t batch = 16;
    // Y: the diagonals over all nE limbs (64-bit words), X: the q limbs'
    // coefficient form, Xp: the special limbs
    u64 *Y = scratch(c, batch * ew), *X = scratch(c, batch * lw), *Xp = scratch(c, batch * pw);
    for (size_t d0 = 0; d0 < nd; d0 += batch) {
        const int nb = (int)std::min(batch, nd - d0);
        frk::db_unpack(c, X, db->data + d0 * db->stride, db->stride, db->lay, L1, nb);
        FR_HIP(hipMemcpy2DAsync(Y, ew * 8, X, lw * 8, lw * 8, nb, hipMemcpyDeviceToDevice, c->stream));
        frk::mont_scale(c, X, L1, qmap(), nb, lw, false);
        frk::ntt_inv(c, X, L1, qmap(), nb, lw);
        if (int e = frk::crt_extend(c, Xp, X, l, nb, pw, lw)) return e;
        frk::ntt_fwd(c, Xp, nP, pmap(c), nb, pw);
        frk::mont_scale(c, Xp, nP, pmap(c), nb, pw, true);
        FR_HIP(hipMemcpy2DAsync(Y + lw, ew * 8, Xp, pw * 8, pw * 8, nb, hipMemcpyDeviceToDevice, c->stream));
        frk::db_pack(c, ext + d0 * stride, stride, lay, Y, nE, nb);
    }
    FR_HIP(hipStreamSynchronize(c->stream));
    (void)hipFree(db->data);
    db->data = ext;
    ext = nullptr;
    db->nl = nE;
    db->stride = stride;
    db->lay = lay;
    return FR_OK;
} FR_CATCH(c)

// out (np polynomials of l limbs) = Rescale(ModDown(U)) for np polynomials
// U over Q_l U P (eval domain, nE limbs each; np even)
// out[p] = Rescale(ModDown(U[p])) for np polynomials over Q_l U P (U items
// su words apart, default nE N; out items so apart, default l N)
static void moddown_rescale(fr_ctx *c, const u64 *U, int np, int l, u64 *out, size_t su = 0, size_t so = 0) {
    Scope sc(c->arena);
    const int N = c->N, nE = l + 1 + c->nP;
    const size_t ew = (size_t)nE * N, lw = (size_t)l * N;
    if (!su) su = ew;
    if (!so) so = lw;
    if (relin_folds(c)) {
        // the top limb and the P limbs in coefficient form drive one forward
        // transform of l limbs whose last pass writes the result
        u64 *Xu = scratch(c, (size_t)np * ew);
        LimbMap top_and_p{l, INT_MAX, 0, l + 1, c->L + 1};
        frk::ntt_inv(c, Xu, c->nP + 1, top_and_p, np, ew, U, su);
        u64 *Z = scratch(c, (size_t)np * lw);
        frk::relin_rescale_prep(c, Z, Xu, nullptr, l, np, lw, ew, 0, true);
        frk::ntt_fwd_relin_rescale(c, Z, l, np, U, su, nullptr, 0, out, so);
        return;
    }
    // other rings: the ciphertext steps on a contiguous copy (an odd count
    // takes a copy of its last polynomial as the partner of that one)
    const int nc = (np + 1) / 2;
    u64 *Uc = scratch(c, (size_t)2 * nc * ew);
    (void)hipMemcpy2DAsync(Uc, ew * 8, U, su * 8, ew * 8, np, hipMemcpyDeviceToDevice, c->stream);
    if (np & 1)
        (void)hipMemcpyAsync(Uc + (size_t)np * ew, U + (size_t)(np - 1) * su, ew * 8, hipMemcpyDeviceToDevice,
                             c->stream);
    u64 *T = scratch(c, (size_t)2 * nc * (l + 1) * N);
    ks_moddown_into(c, Uc, nc, l, T, (size_t)(l + 1) * N, false);
    u64 *O = scratch(c, (size_t)2 * nc * lw);
    rescale_dev(c, T, l, O, nc);
    (void)hipMemcpy2DAsync(out, so * 8, O, lw * 8, lw * 8, np, hipMemcpyDeviceToDevice, c->stream);
}

// Queries q against group groups[q] of extended databases dbs[q] (one ell,
// n1 and level, the queries' level).  Per chunk of queries: one ModUp of
// every c1, the baby steps B_i = (P sigma_i(c0) + U0_i, U1_i) over Q_l U P
// (no ModDown), the inner sums over Q_l U P in one MAC pass, one merged
// ModDown + rescale per inner sum, then the giant steps.
static int matvec_hoisted_impl(fr_ctx *c, const fr_keys *K, const fr_ct *qs, int nq, const fr_db *const *dbs,
                               const int32_t *groups, fr_ct *out) {
    if (int e = keys_ok(c, K, "fr_bsgs_matvec_hoisted")) return e;
    const fr_db *db0 = dbs[0];
    CHECK(db0, FR_EINVAL, "fr_bsgs_matvec_hoisted: null database");
    const int N = c->N, l = db0->level, L1 = l + 1, nE = L1 + c->nP, n1 = db0->n1, ell = db0->ell;
    for (int q = 0; q < nq; ++q) {
        const fr_db *db = dbs[q];
        if (int e = db_ok(c, db, "fr_bsgs_matvec_hoisted")) return e;
        CHECK(db->nl == db->level + 1 + c->nP, FR_EINVAL,
              "fr_bsgs_matvec_hoisted: database not extended to the special primes (fr_db_extend)");
        CHECK(db->ell == ell && db->level == l && db->n1 == n1, FR_EINVAL,
              "fr_bsgs_matvec_hoisted_batch: databases differ in ell, n1 or level");
        CHECK(groups[q] >= 0 && groups[q] < db->G, FR_EINVAL, "fr_bsgs_matvec_hoisted: group %d out of range",
              groups[q]);
        if (int e = check_ct(c, &qs[q], "fr_bsgs_matvec_hoisted")) return e;
        CHECK(qs[q].level == l, FR_ELEVEL, "fr_bsgs_matvec_hoisted: query level %d differs from the database's %d",
              qs[q].level, l);
    }
    CHECK(l >= 1, FR_ELEVEL, "fr_bsgs_matvec_hoisted: no level left to rescale");
    const int n2 = (ell + n1 - 1) / n1;
    for (int i = 1; i < n1; ++i)
        CHECK(K->find(galois_element(N, i)), FR_ENOKEY, "fr_bsgs_matvec_hoisted: no key for baby step %d", i);
    for (int j = 1; j < n2; ++j)
        CHECK(K->find(galois_element(N, j * n1)), FR_ENOKEY, "fr_bsgs_matvec_hoisted: no key for giant step %d",
              j * n1);
    for (int q = 0; q < nq; ++q) {
        if (int e = check_out(c, &out[q], l - 1, "fr_bsgs_matvec_hoisted")) return e;
        for (int t = 0; t < nq; ++t)
            CHECK(out[q].data != qs[t].data, FR_EINVAL, "fr_bsgs_matvec_hoisted: output aliases a query");
    }
    const size_t lw = (size_t)L1 * N, bw = (size_t)2 * nE * N, bq = (size_t)n1 * bw, pw = bw;
    const int ndig = num_digits(c, l);
    const size_t dstride = (size_t)ndig * nE * N;
    auto diag_of = [&](int q) { return (const unsigned char *)(dbs[q]->data + (size_t)groups[q] * ell * dbs[q]->stride); };
    std::vector<int> order(nq);
    for (int q = 0; q < nq; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return diag_of(a) < diag_of(b); });
    const int chunk = c->tune[FR_TUNE_MATVEC_CHUNK];
    for (int q0 = 0; q0 < nq; q0 += chunk) {
        Scope sc(c->arena);
        const int qn = std::min(chunk, nq - q0);
        // the chunk's queries staged contiguously: [qn][2][l+1][N] (read
        // only; a single query is read in place)
        u64 *C = qn == 1 ? qs[order[q0]].data : scratch(c, (size_t)qn * 2 * lw);
        if (qn > 1)
            for (int qq = 0; qq < qn; ++qq)
                FR_HIP(hipMemcpyAsync(C + qq * 2 * lw, qs[order[q0 + qq]].data, 2 * lw * 8, hipMemcpyDeviceToDevice,
                                      c->stream));
        u64 *D = scratch(c, (size_t)qn * dstride);
        ks_modup(c, C + lw, l, D, qn, 2 * lw);
        // inner sums over Q_l U P: [qn][n2][2][nE][N]
        u64 *P = scratch(c, (size_t)qn * n2 * pw);
        std::vector<const unsigned char *> dp(qn);
        for (int qq = 0; qq < qn; ++qq) dp[qq] = diag_of(order[q0 + qq]);
        const bool fused = c->tune[FR_TUNE_KSMAC] > (qn > 1 ? 1 : 0) && frk::bsgs_ksmac_ok(c, l, n1, ell, db0->lay);
        if (fused) {
            // every baby step formed inside the MAC: step 0 from the query,
            // the others from the digit set, c0 and their keys
            std::vector<const unsigned char *> kp(n1);
            std::vector<u64> gp(n1, 1);
            for (int i = 1; i < n1; ++i) {
                gp[i] = galois_element(N, i);
                kp[i] = K->find(gp[i])->data;
            }
            frk::bsgs_ksmac(c, P, (size_t)n2 * pw, qn, n1, dp.data(), db0->stride, db0->lay, D, dstride, C, 2 * lw,
                            kp.data(), gp.data(), l);
        }
        if (!fused) {
            // baby steps over Q_l U P: [qn][n1][2][nE][N]
            u64 *Bb = scratch(c, (size_t)qn * bq);
            frk::scale_ext(c, Bb, C, l, qn, bq, 2 * lw);
            if (frk::ks_inner_multi_ok(c, l)) {
                // every baby step from one read of the digit set and of c0
                std::vector<const unsigned char *> kp(n1 - 1);
                std::vector<u64> gp(n1 - 1);
                for (int i = 1; i < n1; ++i) {
                    gp[i - 1] = galois_element(N, i);
                    kp[i - 1] = K->find(gp[i - 1])->data;
                }
                frk::ks_inner_multi(c, Bb + bw, bw, D, kp.data(), gp.data(), n1 - 1, l, qn, dstride, bq, C, 2 * lw);
            } else {
                for (int i = 1; i < n1; ++i) {
                    const u64 g = galois_element(N, i);
                    u64 *Ui = Bb + i * bw;
                    frk::ks_inner(c, Ui, Ui + (size_t)nE * N, D, K->find(g)->data, g, l, false, qn, dstride, bq,
                                  nullptr, 0, C, 2 * lw);
                }
            }
            std::vector<const u64 *> bp((size_t)qn * n1);
            for (int qq = 0; qq < qn; ++qq)
                for (int i = 0; i < n1; ++i) bp[(size_t)qq * n1 + i] = Bb + qq * bq + i * bw;
            frk::bsgs_mac(c, P, (size_t)n2 * pw, bp.data(), qn, n1, dp.data(), db0->stride, db0->lay, ell, nE - 1,
                          nE - 1, l, c->L - l);
        }
        // a rotation needs no key for an inner sum's first polynomial: those
        // are rotated and summed over Q_l U P (Asum, one per query) and take
        // one ModDown + rescale together; every second polynomial takes its
        // own, for its key switch in the giant steps
        u64 *Asum = scratch(c, (size_t)qn * nE * N);
        std::vector<u64> gj(n2);
        for (int j = 0; j < n2; ++j) gj[j] = galois_element(N, j * n1);
        frk::automorph_sum(c, Asum, P, gj.data(), n2, nE, qn, (size_t)nE * N, pw, (size_t)n2 * pw, l, false);
        // R = [qn][n2][2][l][N]: R_{q,j}.c1 for every j, and R_{q,0}.c0 the sum
        u64 *R = scratch(c, (size_t)qn * n2 * 2 * l * N);
        moddown_rescale(c, P + (size_t)nE * N, qn * n2, l, R + (size_t)l * N, pw, (size_t)2 * l * N);
        moddown_rescale(c, Asum, qn, l, R, (size_t)nE * N, (size_t)n2 * 2 * l * N);
        std::vector<u64 *> op(qn);
        for (int qq = 0; qq < qn; ++qq) op[qq] = out[order[q0 + qq]].data;
        if (int e = giant_steps(c, K, R, qn, n2, n1, l - 1, op.data(), true)) return e;
    }
    FR_HIP(hipGetLastError());
    for (int q = 0; q < nq; ++q) {
        out[q].level = l - 1;
        out[q].scale = (qs[q].scale * dbs[q]->scale) / (double)c->mod[l];
    }
    return FR_OK;
}

extern "C" int fr_bsgs_matvec_hoisted(fr_ctx *c, const fr_keys *K, const fr_ct *query, const fr_db *db, int32_t group,
                                      fr_ct *out) try {
    CHECK(c && K && query && db && out, FR_EINVAL, "fr_bsgs_matvec_hoisted: null argument");
    c->arena.reset();
    return matvec_hoisted_impl(c, K, query, 1, &db, &group, out);
} FR_CATCH(c)

extern "C" int fr_bsgs_matvec_hoisted_batch(fr_ctx *c, const fr_keys *K, const fr_ct *queries, int32_t nq,
                                            const fr_db *const *dbs, const int32_t *groups, fr_ct *out) try {
    CHECK(c && K && queries && dbs && groups && out && nq >= 1, FR_EINVAL,
          "fr_bsgs_matvec_hoisted_batch: null argument or empty batch");
    c->arena.reset();
    return matvec_hoisted_impl(c, K, queries, nq, dbs, groups, out);
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// parity hook: the device ModDown paths on caller-given residues
// ---------------------------------------------------------------------------
extern "C" int fr_moddown_parity(fr_ctx *c, int32_t mode, const uint64_t *u_host, const uint64_t *d_host,
                                 int32_t level, fr_ct *out) try {
    if (c) if (int e_ = no_capture(c, "fr_moddown_parity")) return e_;
    CHECK(c && u_host && out, FR_EINVAL, "fr_moddown_parity: null argument");
    CHECK(mode >= 0 && mode <= 2, FR_EINVAL, "fr_moddown_parity: unknown mode %d", mode);
    CHECK(mode != 2 || d_host, FR_EINVAL, "fr_moddown_parity: mode 2 needs d");
    CHECK(level >= (mode ? 1 : 0) && level <= c->L, FR_ELEVEL, "fr_moddown_parity: bad level %d", level);
    const int ol = mode ? level - 1 : level;
    if (int e = check_out(c, out, ol, "fr_moddown_parity")) return e;
    const int N = c->N, nE = level + 1 + c->nP;
    const size_t ew = (size_t)nE * N, lw = (size_t)(level + 1) * N;
    std::vector<u64> hu(u_host, u_host + 2 * ew);
    for (int p = 0; p < 2; ++p)
        for (int e = 0; e < nE; ++e) {
            const u64 q = c->mod[e <= level ? e : c->L + 1 + (e - level - 1)];
            for (int k = 0; k < N; ++k)
                CHECK(hu[(size_t)p * ew + (size_t)e * N + k] < q, FR_EINVAL,
                      "fr_moddown_parity: residue not canonical (limb %d)", e);
        }
    c->arena.reset();
    Scope sc(c->arena);
    u64 *U = scratch(c, 2 * ew);
    u64 *d = mode == 2 ? scratch(c, 2 * lw) : nullptr;
    CHECK(U && (mode != 2 || d), FR_ENOMEM, "fr_moddown_parity: scratch");
    const LimbMap ext{0, INT_MAX, 0, level + 1, c->L + 1};
    FR_HIP(hipMemcpyAsync(U, hu.data(), 2 * ew * 8, hipMemcpyHostToDevice, c->stream));
    frk::ntt_fwd(c, U, nE, ext, 2, ew);
    if (mode == 2) {
        for (int p = 0; p < 2; ++p)
            for (int i = 0; i <= level; ++i)
                for (int k = 0; k < N; ++k)
                    CHECK(d_host[(size_t)p * lw + (size_t)i * N + k] < c->mod[i], FR_EINVAL,
                          "fr_moddown_parity: d residue not canonical (limb %d)", i);
        FR_HIP(hipMemcpyAsync(d, d_host, 2 * lw * 8, hipMemcpyHostToDevice, c->stream));
        frk::ntt_fwd(c, d, level + 1, qmap(), 2, lw);
    }
    if (mode == 0) {
        ks_moddown(c, U, level, out->data, false);
    } else if (mode == 1) {
        moddown_rescale(c, U, 2, level, out->data);
    } else {
        // the relinearised product's path: the key inner product leaves
        // d_l + P^-1 U_l in U's top limb where the merged step expects it
        if (relin_folds(c)) frk::fold_top(c, U, d, level, 2, ew, lw);
        relin_rescale_into(c, d, U, 1, level, out->data);
    }
    FR_HIP(hipGetLastError());
    FR_HIP(hipStreamSynchronize(c->stream));
    out->level = ol;
    out->scale = 1.0;
    return FR_OK;
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// Chebyshev threshold
// ---------------------------------------------------------------------------
// The recursion is written once (Cheb<B>) and run on a recording backend that
// builds the DAG of operations: Chebyshev-basis division p = q T_M + r
// (q_0 = c_M, q_i = 2 c_{M+i}, r_0 = c_0, r_k = c_k - c_{2M-k}) with M = d1 2^j
// the largest below the number of coefficients, leaves of at most d1
// coefficients, and powers T_i = 2 T_ceil(i/2) T_floor(i/2) - T_(i mod 2).
// The DAG gives the planning answers (levels, product count) and is executed
// on the device in waves: every operation whose inputs are ready runs in the
// same wave, relinearised products and rescales of one wave in one batch.
namespace {

enum COp { C_INPUT, C_ADJUST, C_MUL, C_ADD, C_SUB, C_TWICE_M1, C_TWICE_SUB, C_SCALAR, C_LEAF };

struct CNode {
    COp op;
    int a = -1, b = -1;
    int level = 0;
    double cst = 0.0;
    std::vector<int> ins;    // leaf: T_1..T_{m-1}
    std::vector<double> cf;  // leaf: c_0..c_{m-1}
};

struct RH {
    int id = -1;
    explicit operator bool() const { return id >= 0; }
};

struct Recorder {
    using H = RH;
    std::vector<CNode> nodes;
    int nmul = 0;
    bool fail = false;
    H push(CNode n) {
        nodes.push_back(std::move(n));
        return H{(int)nodes.size() - 1};
    }
    H input(int level) {
        CNode n{C_INPUT};
        n.level = level;
        return push(n);
    }
    int level(const H &h) const { return nodes[h.id].level; }
    H adjust(const H &a, int lam) {
        if (!a) return H();
        if (level(a) == lam) return a;
        if (lam < 0 || lam > level(a)) {
            fail = true;
            return H();
        }
        CNode n{C_ADJUST};
        n.a = a.id;
        n.level = lam;
        return push(n);
    }
    H mul(const H &a, const H &b) {
        if (!a || !b) return H();
        const int lam = std::min(level(a), level(b));
        if (lam < 1) {
            fail = true;
            return H();
        }
        H x = adjust(a, lam), y = adjust(b, lam);
        CNode n{C_MUL};
        n.a = x.id;
        n.b = y.id;
        n.level = lam - 1;
        ++nmul;
        return push(n);
    }
    H bin(COp op, const H &a, const H &b) {
        if (!a || !b) return H();
        CNode n{op};
        n.a = a.id;
        n.b = b.id;
        n.level = level(a);
        return push(n);
    }
    H add(const H &a, const H &b) { return bin(C_ADD, a, b); }
    H sub(const H &a, const H &b) { return bin(C_SUB, a, b); }
    H twice_sub(const H &a, const H &b) { return bin(C_TWICE_SUB, a, b); }  // 2 a - b
    H twice_minus_const(const H &a) {
        if (!a) return H();
        CNode n{C_TWICE_M1};
        n.a = a.id;
        n.level = level(a);
        return push(n);
    }
    H scalar(const H &T, double cst) {
        if (!T) return H();
        if (level(T) < 1) {
            fail = true;
            return H();
        }
        CNode n{C_SCALAR};
        n.a = T.id;
        n.cst = cst;
        n.level = level(T) - 1;
        return push(n);
    }
    H leaf(const std::vector<H> &Ts, const double *cf, int m) {
        int lam = INT_MAX;
        CNode n{C_LEAF};
        for (int i = 1; i < m; ++i) {
            if (!Ts[i]) return H();
            lam = std::min(lam, level(Ts[i]) - 1);
            n.ins.push_back(Ts[i].id);
        }
        if (lam < 0) {
            fail = true;
            return H();
        }
        n.cf.assign(cf, cf + m);
        n.level = lam;
        return push(n);
    }
};

template <class B>
struct Cheb {
    B &be;
    int d1;
    std::vector<typename B::H> T;
    using H = typename B::H;

    H power(int i) {
        if (T[i]) return T[i];
        const int a = (i + 1) / 2, b = i / 2;
        H Ta = power(a), Tb = power(b);
        if (be.fail || !Ta || !Tb) return H();
        H prod = be.mul(Ta, Tb);
        if (!prod) return H();
        H res;
        if (a == b) {
            res = be.twice_minus_const(prod);
        } else {
            // 2 T_a T_b - T_1 in one pass (the same words as a doubling and a subtraction)
            H t1 = be.adjust(T[1], be.level(prod));
            res = be.twice_sub(prod, t1);
        }
        T[i] = res;
        return res;
    }

    H eval(const std::vector<double> &cf, int m) {
        if (be.fail) return H();
        if (m <= d1) {
            for (int i = 1; i < m; ++i)
                if (!power(i)) return H();
            return be.leaf(T, cf.data(), m);
        }
        int M = d1;
        while (2 * M < m) M *= 2;
        const int nq = m - M;
        std::vector<double> q(nq), r(M);
        q[0] = cf[M];
        for (int i = 1; i < nq; ++i) q[i] = 2.0 * cf[M + i];
        r[0] = cf[0];
        for (int k = 1; k < M; ++k) r[k] = cf[k] - ((2 * M - k < m) ? cf[2 * M - k] : 0.0);
        H TM = power(M);
        if (!TM) return H();
        H A;
        if (nq == 1) {
            A = be.scalar(TM, q[0]);
        } else {
            H Q = eval(q, nq);
            if (!Q) return H();
            A = be.mul(Q, TM);
        }
        if (!A) return H();
        H R = eval(r, M);
        if (!R) return H();
        const int lam = std::min(be.level(A), be.level(R));
        H x = be.adjust(A, lam), y = be.adjust(R, lam);
        return be.add(x, y);
    }
};

// records the evaluation of a degree-`degree` series from an input at in_level
struct ChebPlan {
    Recorder rec;
    RH out;
    bool ok = false;
    ChebPlan(int in_level, const double *cf, int degree, int d1) {
        Cheb<Recorder> ch{rec, d1, std::vector<RH>(std::max(degree + 2, 2 * d1 + 2))};
        ch.T[1] = rec.input(in_level);
        std::vector<double> coef(cf, cf + degree + 1);
        out = ch.eval(coef, degree + 1);
        ok = out && !rec.fail;
    }
};

long long rne_ll(double x) { return (long long)std::nearbyint(x); }

// Executes the recorded DAG in waves for nq inputs at once (the same DAG for
// every query).  Node outputs live in the arena for the duration of the call
// (buf[node * nq + q]); every ciphertext of a wave that needs a rescale is
// staged contiguously so that one batched rescale serves the wave.
int cheb_execute(fr_ctx *c, const fr_keys *K, const std::vector<CNode> &nodes, const double *D,
                 const u64 *const *in, int nq, std::vector<u64 *> &buf) {
    const int N = c->N, n = (int)nodes.size();
    std::vector<int> depth(n, 0);
    int maxd = 0;
    for (int i = 0; i < n; ++i) {
        const CNode &nd = nodes[i];
        int d = 0;
        if (nd.a >= 0) d = std::max(d, depth[nd.a] + 1);
        if (nd.b >= 0) d = std::max(d, depth[nd.b] + 1);
        for (int x : nd.ins) d = std::max(d, depth[x] + 1);
        depth[i] = d;
        maxd = std::max(maxd, d);
    }
    // Critical-first schedule: tail[i] estimates the time from node i's
    // start to the output along its longest chain of consumers (per-node
    // costs in microseconds of one query: a relinearised product about 200,
    // a scalar wave with its rescale about 80, an addition about 12).  A
    // level adjustment or scalar multiple moves to the depth just before its
    // first consumer, where it no longer shares a wave (and its rescale) with
    // the leaves of the critical chain; its inputs come from earlier depths
    // still.  Nodes are recorded after their inputs, so consumers have the
    // larger indices.
    const bool crit = c->tune[FR_TUNE_CHEB_SCHED] != 0;
    std::vector<int> tail(n, 0);
    if (crit) {
        std::vector<std::vector<int>> cons(n);
        for (int i = 0; i < n; ++i) {
            const CNode &nd = nodes[i];
            if (nd.a >= 0) cons[nd.a].push_back(i);
            if (nd.b >= 0 && nd.b != nd.a) cons[nd.b].push_back(i);
            for (int x : nd.ins) cons[x].push_back(i);
        }
        for (int i = n - 1; i >= 0; --i) {
            const COp op = nodes[i].op;
            const int cost = op == C_MUL ? 200 : (op == C_ADJUST || op == C_SCALAR || op == C_LEAF) ? 80
                                                 : op == C_INPUT ? 0 : 12;
            int t = 0, dl = INT_MAX;
            for (int j : cons[i]) {
                t = std::max(t, tail[j]);
                dl = std::min(dl, depth[j] - 1);
            }
            tail[i] = t + cost;
            if ((op == C_ADJUST || op == C_SCALAR) && dl != INT_MAX) depth[i] = dl;
        }
    }
    buf.assign((size_t)n * nq, nullptr);
    auto B_ = [&](int node, int q) -> u64 *& { return buf[(size_t)node * nq + q]; };
    for (int i = 0; i < n; ++i)
        if (nodes[i].op == C_INPUT)
            for (int q = 0; q < nq; ++q) B_(i, q) = const_cast<u64 *>(in[q]);
    const KeyEntry *rk = K->find(0);
    CHECK(rk, FR_ENOKEY, "fr_chebyshev_eval: relinearisation key missing");
    auto lw = [&](int level) { return (size_t)(level + 1) * N; };
    // The groups of one depth (scalar family, products and additions, each
    // per level) depend only on earlier depths.  They are spread over the
    // caller's stream and the auxiliary streams; a group waits only for the
    // groups that produced its inputs (an event recorded after each group),
    // and every stream is joined into the caller's at the end.  Arena space
    // is not reused inside the call, so no group's scratch is handed to
    // another stream.
    c->arena.hold++;
    struct HoldGuard {
        Arena &a;
        ~HoldGuard() { a.hold--; }
    } hold_guard{c->arena};
    const hipStream_t main_stream = c->stream;
    StreamRestore restore(c->stream);
    const int nstream = 1 + fr_ctx::kAux;
    auto stream_of = [&](int s) { return s == 0 ? main_stream : c->aux[s - 1]; };
    // event slot, stream and issue order of the group that produced each node
    std::vector<int> prod_ev(n, -1), prod_st(n, 0), prod_seq(n, -1);
    constexpr int kSlots = fr_ctx::kDagEv / (1 + fr_ctx::kAux);
    int ev_next[1 + fr_ctx::kAux] = {}, rr = 0, seq = 0;
    bool aux_used = false;
    FR_HIP(hipEventRecord(c->ev_fork, main_stream));  // the inputs, for the auxiliary streams
    for (int d = 1; d <= maxd; ++d) {
        std::vector<std::function<int()>> groups;
        std::vector<std::vector<int>> gin, gout;  // input and output nodes of each group
        // --- scalar family (adjust, scalar, leaf), grouped by output level
        std::vector<std::vector<int>> by_level(FR_MAXLEVEL), mul_by_level(FR_MAXLEVEL);
        for (int i = 0; i < n; ++i) {
            if (depth[i] != d) continue;
            const COp op = nodes[i].op;
            if (op == C_ADJUST || op == C_SCALAR || op == C_LEAF) by_level[nodes[i].level].push_back(i);
            if (op == C_MUL) mul_by_level[nodes[i].level + 1].push_back(i);
        }
        for (int lam = 0; lam < FR_MAXLEVEL; ++lam) {
            if (by_level[lam].empty()) continue;
            gout.push_back(by_level[lam]);
            gin.emplace_back();
            for (int i : by_level[lam]) {
                const CNode &nd = nodes[i];
                if (nd.op == C_ADJUST || nd.op == C_SCALAR) gin.back().push_back(nd.a);
                else gin.back().insert(gin.back().end(), nd.ins.begin(), nd.ins.end());
            }
            groups.push_back([&, lam]() -> int {
                const auto &L = by_level[lam];
                const int B = (int)L.size() * nq;  // item b = node L[b / nq], query b % nq
                const size_t sw = 2 * lw(lam + 1), ow = 2 * lw(lam);
                u64 *stage = scratch(c, (size_t)B * sw);
                u64 *out = scratch(c, (size_t)B * ow);
                // the integer terms (source node, k) of every node of the wave
                const int nL = (int)L.size();
                std::vector<std::vector<std::pair<int, long long>>> terms(nL);
                std::vector<long long> cst(B, 0);
                bool any_const = false;
                for (int j = 0; j < nL; ++j) {
                    const CNode &nd = nodes[L[j]];
                    if (nd.op == C_ADJUST || nd.op == C_SCALAR) {
                        const int la = nodes[nd.a].level;
                        const long long k = nd.op == C_ADJUST
                                                ? rne_ll((D[lam] * (double)c->mod[lam + 1]) / D[la])
                                                : rne_ll(((nd.cst * D[lam]) * (double)c->mod[la]) / D[la]);
                        terms[j].push_back({nd.a, k});
                    } else {
                        for (size_t t = 0; t < nd.ins.size(); ++t) {
                            const int src = nd.ins[t], ls = nodes[src].level;
                            terms[j].push_back(
                                {src, rne_ll(((nd.cf[t + 1] * D[lam]) * (double)c->mod[lam + 1]) / D[ls])});
                        }
                        for (int q = 0; q < nq; ++q) cst[j * nq + q] = rne_ll(nd.cf[0] * D[lam]);
                        any_const = true;
                    }
                }
                // every source of the wave read once for all its outputs when
                // they are few, else item by item
                std::vector<int> su;
                for (auto &tj : terms)
                    for (auto &t : tj)
                        if (std::find(su.begin(), su.end(), t.first) == su.end()) su.push_back(t.first);
                const int ns = (int)su.size();
                std::vector<long long> Km((size_t)nL * ns, 0);
                std::vector<int> slp1(ns);
                std::vector<const u64 *> sp((size_t)nq * ns);
                for (int s = 0; s < ns; ++s) {
                    slp1[s] = nodes[su[s]].level + 1;
                    for (int q = 0; q < nq; ++q) sp[(size_t)q * ns + s] = B_(su[s], q);
                }
                for (int j = 0; j < nL; ++j)
                    for (auto &t : terms[j]) {
                        const int s = (int)(std::find(su.begin(), su.end(), t.first) - su.begin());
                        Km[(size_t)j * ns + s] += t.second;
                    }
                if (!frk::scalar_mat(c, stage, lam + 2, nL, nq, sp.data(), slp1.data(), ns, Km.data(), nq * sw, sw)) {
                    std::vector<ScalarItem> items(B);
                    for (int b = 0; b < B; ++b)
                        for (auto &t : terms[b / nq]) {
                            items[b].src.push_back(B_(t.first, b % nq));
                            items[b].k.push_back(t.second);
                            items[b].lp1.push_back(nodes[t.first].level + 1);
                        }
                    frk::scalar_batch(c, stage, lam + 2, B, items.data());
                }
                rescale_dev(c, stage, lam + 1, out, B);
                if (any_const) frk::add_const_batch(c, out, lam + 1, B, cst.data(), ow);
                for (int b = 0; b < B; ++b) B_(L[b / nq], b % nq) = out + (size_t)b * ow;
                return FR_OK;
            });
        }
        // --- relinearised products, grouped by input level
        for (int lv = 1; lv < FR_MAXLEVEL; ++lv) {
            if (mul_by_level[lv].empty()) continue;
            gout.push_back(mul_by_level[lv]);
            gin.emplace_back();
            for (int i : mul_by_level[lv]) {
                gin.back().push_back(nodes[i].a);
                gin.back().push_back(nodes[i].b);
            }
            groups.push_back([&, lv]() -> int {
                const auto &L = mul_by_level[lv];
                const int B = (int)L.size() * nq, nE = lv + 1 + c->nP, ndig = num_digits(c, lv);
                const size_t cw = 2 * lw(lv);
                u64 *T01 = scratch(c, (size_t)B * cw);
                u64 *T2 = scratch(c, (size_t)B * lw(lv));
                u64 *Dg = scratch(c, (size_t)B * ndig * nE * N);
                u64 *U = scratch(c, (size_t)B * 2 * nE * N);
                u64 *out = scratch(c, (size_t)B * 2 * lw(lv - 1));
                std::vector<const u64 *> xa(B), yb(B);
                for (int b = 0; b < B; ++b) {
                    xa[b] = B_(nodes[L[b / nq]].a, b % nq);
                    yb[b] = B_(nodes[L[b / nq]].b, b % nq);
                }
                frk::tensor_batch(c, T01, T2, lv + 1, B, xa.data(), yb.data());
                ks_modup(c, T2, lv, Dg, B, lw(lv));
                frk::ks_inner(c, U, U + (size_t)nE * N, Dg, rk->data, 1, lv, false, B, (size_t)ndig * nE * N,
                              (size_t)2 * nE * N, relin_folds(c) ? T01 : nullptr, cw);
                relin_rescale_into(c, T01, U, B, lv, out);
                for (int b = 0; b < B; ++b) B_(L[b / nq], b % nq) = out + (size_t)b * 2 * lw(lv - 1);
                return FR_OK;
            });
        }
        // --- additions, grouped by level
        for (int lv = 0; lv < FR_MAXLEVEL; ++lv) {
            std::vector<int> L;
            for (int i = 0; i < n; ++i) {
                const COp op = nodes[i].op;
                if (depth[i] == d && nodes[i].level == lv &&
                    (op == C_ADD || op == C_SUB || op == C_TWICE_M1 || op == C_TWICE_SUB))
                    L.push_back(i);
            }
            if (L.empty()) continue;
            gout.push_back(L);
            gin.emplace_back();
            for (int i : L) {
                gin.back().push_back(nodes[i].a);
                if (nodes[i].op != C_TWICE_M1) gin.back().push_back(nodes[i].b);
            }
            groups.push_back([&, lv, L]() -> int {
                const int B = (int)L.size() * nq;
                const size_t w = lw(lv);
                u64 *o = scratch(c, (size_t)B * 2 * w);
                std::vector<const u64 *> xa(B), yb(B);
                std::vector<u64 *> outs(B);
                std::vector<long long> cst(B, 0);
                std::vector<int> op(B, 0);
                for (int b = 0; b < B; ++b) {
                    const CNode &nd = nodes[L[b / nq]];
                    const int q = b % nq;
                    xa[b] = B_(nd.a, q);
                    yb[b] = nd.op == C_TWICE_M1 ? B_(nd.a, q) : B_(nd.b, q);
                    outs[b] = o + (size_t)b * 2 * w;
                    op[b] = nd.op == C_SUB ? 1 : nd.op == C_TWICE_SUB ? 2 : 0;
                    if (nd.op == C_TWICE_M1) cst[b] = rne_ll(-1.0 * D[lv]);
                }
                frk::pair_batch(c, lv + 1, B, xa.data(), yb.data(), outs.data(), cst.data(), op.data());
                for (int b = 0; b < B; ++b) B_(L[b / nq], b % nq) = outs[b];
                return FR_OK;
            });
        }
        // each group on the stream of its most recently issued input (that
        // input's producer is the likeliest to finish last, and a wait on
        // the group's own stream costs nothing), unless another group of this
        // depth took that stream already; else on the next free stream in
        // turn.  It waits for the events of the groups on other streams that
        // produced its inputs.
        // issue order: as built, or (critical-first) longest tail first
        std::vector<int> order(groups.size());
        for (size_t g = 0; g < groups.size(); ++g) order[g] = (int)g;
        if (crit) {
            std::vector<int> prio(groups.size(), 0);
            for (size_t g = 0; g < groups.size(); ++g)
                for (int x : gout[g]) prio[g] = std::max(prio[g], tail[x]);
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return prio[x] > prio[y]; });
        }
        std::vector<char> taken(nstream, 0);
        for (const int g : order) {
            int st = -1, latest = -1;
            for (int x : gin[g])
                if (prod_seq[x] > latest) latest = prod_seq[x], st = prod_st[x];
            if (st < 0 || taken[st]) {
                st = rr % nstream;
                for (int k = 0; k < nstream; ++k)
                    if (!taken[(rr + k) % nstream]) {
                        st = (rr + k) % nstream;
                        break;
                    }
                ++rr;
            }
            taken[st] = 1;
            const hipStream_t s = stream_of(st);
            if (st > 0 && !aux_used) {
                for (int a = 0; a < fr_ctx::kAux; ++a) FR_HIP(hipStreamWaitEvent(c->aux[a], c->ev_fork, 0));
                aux_used = true;
            }
            std::vector<int> waited;
            for (int x : gin[g]) {
                const int ev = prod_ev[x];
                if (ev < 0 || prod_st[x] == st || std::find(waited.begin(), waited.end(), ev) != waited.end())
                    continue;
                FR_HIP(hipStreamWaitEvent(s, c->ev_dag[ev], 0));
                waited.push_back(ev);
            }
            c->stream = s;
            const int e = groups[g]();
            c->stream = main_stream;
            if (e) return e;
            const int ev = st * kSlots + ev_next[st]++ % kSlots;
            FR_HIP(hipEventRecord(c->ev_dag[ev], s));
            for (int x : gout[g]) {
                prod_ev[x] = ev;
                prod_st[x] = st;
                prod_seq[x] = seq;
            }
            ++seq;
        }
    }
    if (aux_used)
        for (int a = 0; a < fr_ctx::kAux; ++a) {
            FR_HIP(hipEventRecord(c->ev_join[a], c->aux[a]));
            FR_HIP(hipStreamWaitEvent(main_stream, c->ev_join[a], 0));
        }
    return FR_OK;
}


int chebyshev_impl(fr_ctx *c, const fr_keys *K, const fr_ct *in, int nq, const double *cf, int degree, int d1,
                   fr_ct *out) {
    if (int e = keys_ok(c, K, "fr_chebyshev_eval")) return e;
    CHECK(degree >= 1 && d1 >= 2, FR_EINVAL, "fr_chebyshev_eval: need degree >= 1 and d1 >= 2");
    for (int q = 0; q < nq; ++q) {
        if (int e = check_ct(c, &in[q], "fr_chebyshev_eval")) return e;
        CHECK(in[q].level == in[0].level && in[q].scale == in[0].scale, FR_ELEVEL,
              "fr_chebyshev_eval_batch: inputs differ in level or scale");
    }
    ChebPlan plan(in[0].level, cf, degree, d1);
    CHECK(plan.ok, FR_ELEVEL, "fr_chebyshev_eval: not enough levels for degree %d from level %d", degree,
          in[0].level);
    const int ol = plan.rec.nodes[plan.out.id].level;
    for (int q = 0; q < nq; ++q)
        if (int e = check_out(c, &out[q], ol, "fr_chebyshev_eval")) return e;
    CHECK(K->find(0), FR_ENOKEY, "fr_chebyshev_eval: relinearisation key missing");
    double D[FR_MAXLEVEL];
    D[in[0].level] = in[0].scale;
    for (int l = in[0].level; l >= 1; --l) D[l - 1] = (D[l] * D[l]) / (double)c->mod[l];
    const size_t ow = (size_t)2 * (ol + 1) * c->N;
    // queries per pass (bounds the arena: every node output of the pass
    // stays live until the pass ends)
    const int chunk = c->tune[FR_TUNE_CHEB_CHUNK];
    for (int q0 = 0; q0 < nq; q0 += chunk) {
        const int qn = std::min(chunk, nq - q0);
        c->arena.reset();
        Scope sc(c->arena);
        std::vector<const u64 *> ip(qn);
        for (int q = 0; q < qn; ++q) ip[q] = in[q0 + q].data;
        std::vector<u64 *> buf;
        if (int e = cheb_execute(c, K, plan.rec.nodes, D, ip.data(), qn, buf)) return e;
        for (int q = 0; q < qn; ++q)
            FR_HIP(hipMemcpyAsync(out[q0 + q].data, buf[(size_t)plan.out.id * qn + q], ow * 8,
                                  hipMemcpyDeviceToDevice, c->stream));
    }
    FR_HIP(hipGetLastError());
    for (int q = 0; q < nq; ++q) {
        out[q].level = ol;
        out[q].scale = D[ol];
    }
    return FR_OK;
}

}  // namespace

extern "C" int fr_chebyshev_eval(fr_ctx *c, const fr_keys *K, const fr_ct *in, const double *cf, int32_t degree,
                                 int32_t d1, fr_ct *out) try {
    CHECK(c && K && in && cf && out, FR_EINVAL, "fr_chebyshev_eval: null argument");
    return chebyshev_impl(c, K, in, 1, cf, degree, d1, out);
} FR_CATCH(c)

extern "C" int fr_chebyshev_eval_batch(fr_ctx *c, const fr_keys *K, const fr_ct *in, int32_t nq, const double *cf,
                                       int32_t degree, int32_t d1, fr_ct *out) try {
    CHECK(c && K && in && cf && out && nq >= 1, FR_EINVAL, "fr_chebyshev_eval_batch: null argument or empty batch");
    return chebyshev_impl(c, K, in, nq, cf, degree, d1, out);
} FR_CATCH(c)

extern "C" int fr_cheb_out_level(int32_t in_level, int32_t degree, int32_t d1) {
    if (degree < 1 || d1 < 2 || in_level < 0) return -1;
    std::vector<double> coef(degree + 1, 1.0);
    ChebPlan plan(in_level, coef.data(), degree, d1);
    return plan.ok ? plan.rec.nodes[plan.out.id].level : -1;
}

extern "C" int fr_cheb_mult_count(int32_t degree, int32_t d1) {
    if (degree < 1 || d1 < 2) return -1;
    std::vector<double> coef(degree + 1, 1.0);
    ChebPlan plan(1 << 20, coef.data(), degree, d1);
    return plan.rec.nmul;
}

// ---------------------------------------------------------------------------
// captured call sequences (HIP graphs)
// ---------------------------------------------------------------------------
struct fr_graph {
    fr_ctx *ctx;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned gen = 0;
};

// Capture is switched off: recording the hoisted product and the Chebyshev
// ladder (work forked over the auxiliary streams, 2-D copies) ended in a host
// fault inside hipStreamEndCapture / hipGraphInstantiate whose cause is not
// established.  The recording code below stays for when it is.
static const bool kGraphCapture = false;

extern "C" int fr_graph_begin(fr_ctx *c) try {
    CHECK(c, FR_EINVAL, "null context");
    CHECK(kGraphCapture, FR_EINVAL, "fr_graph_begin: HIP-graph capture is switched off in this library");
    CHECK(!c->capturing, FR_EINVAL, "fr_graph_begin: a capture is already in progress");
    CHECK(!c->prof || c->prof->cls == K_NONE, FR_EINVAL, "fr_graph_begin: the timing hook is active");
    if (!c->cap_stream) FR_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    // the recorded work starts after what the caller's stream already holds
    FR_HIP(hipStreamSynchronize(c->stream));
    FR_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    c->saved_stream = c->stream;
    c->stream = c->cap_stream;
    c->capturing = true;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_graph_end(fr_ctx *c, fr_graph **out) try {
    CHECK(c && out, FR_EINVAL, "fr_graph_end: null argument");
    CHECK(c->capturing, FR_EINVAL, "fr_graph_end: no capture in progress");
    c->stream = c->saved_stream;
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return fr_fail(FR_EHIP, "fr_graph_end: the capture failed (%s); a recorded call may have needed the host",
                       hipGetErrorString(e));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fr_fail(FR_EHIP, "fr_graph_end: instantiate: %s", hipGetErrorString(ei));
    }
    fr_graph *gr = new fr_graph();
    gr->ctx = c;
    gr->graph = g;
    gr->exec = x;
    gr->gen = c->arena_gen;
    *out = gr;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_graph_launch(fr_ctx *c, const fr_graph *g) try {
    CHECK(c && g, FR_EINVAL, "fr_graph_launch: null argument");
    CHECK(g->ctx == c, FR_EINVAL, "fr_graph_launch: graph of another context");
    CHECK(!c->capturing, FR_EINVAL, "fr_graph_launch: a capture is in progress");
    CHECK(g->gen == c->arena_gen, FR_EINVAL, "fr_graph_launch: the context's scratch was released after the capture");
    FR_HIP(hipGraphLaunch(g->exec, c->stream));
    return FR_OK;
} FR_CATCH(c)

extern "C" void fr_graph_destroy(fr_graph *g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->ctx->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

// ---------------------------------------------------------------------------
// kernel timing hook
// ---------------------------------------------------------------------------
bool Prof::begin(int k, hipStream_t s) {
    if (cls != k || 2 * used + 1 >= (int)ev.size()) return false;
    return hipEventRecord(ev[2 * used], s) == hipSuccess;
}
void Prof::end(int, hipStream_t s, double b) {
    (void)hipEventRecord(ev[2 * used + 1], s);
    ++used;
    bytes += b;
}

extern "C" int fr_prof_begin(fr_ctx *c, int32_t kernel_class) try {
    CHECK(c, FR_EINVAL, "null context");
    CHECK(!c->capturing, FR_EINVAL, "fr_prof_begin: a graph capture is in progress");
    CHECK(kernel_class >= 0 && kernel_class <= K_ELEM, FR_EINVAL, "fr_prof_begin: unknown class %d", kernel_class);
    if (!c->prof) {
        c->prof = new Prof();
        c->prof->ev.resize(2 * 16384);
        for (auto &e : c->prof->ev) FR_HIP(hipEventCreate(&e));
    }
    FR_HIP(hipStreamSynchronize(c->stream));
    c->prof->cls = kernel_class;
    c->prof->used = 0;
    c->prof->bytes = 0.0;
    return FR_OK;
} FR_CATCH(c)

extern "C" int fr_prof_end(fr_ctx *c, int32_t *launches, double *total_ms, double *bytes) try {
    CHECK(c && c->prof, FR_EINVAL, "fr_prof_end: no timing in progress");
    FR_HIP(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (int i = 0; i < c->prof->used; ++i) {
        float ms = 0.f;
        FR_HIP(hipEventElapsedTime(&ms, c->prof->ev[2 * i], c->prof->ev[2 * i + 1]));
        tot += ms;
    }
    if (launches) *launches = c->prof->used;
    if (total_ms) *total_ms = tot;
    if (bytes) *bytes = c->prof->bytes;
    c->prof->cls = K_NONE;
    c->prof->used = 0;
    return FR_OK;
} FR_CATCH(c)

// ---------------------------------------------------------------------------
// host-only planning helpers
// ---------------------------------------------------------------------------
extern "C" int fr_cheb_step_coeffs(int32_t degree, double delta, double *c) {
    if (degree < 1 || !c) return fr_fail(FR_EINVAL, "fr_cheb_step_coeffs: bad arguments");
    const int n = degree + 1;
    std::vector<double> f(n), th(n);
    for (int j = 0; j < n; ++j) {
        th[j] = M_PI * ((double)j + 0.5) / (double)n;
        f[j] = std::cos(th[j]) >= delta ? 1.0 : 0.0;
    }
    for (int k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += f[j] * std::cos((double)k * th[j]);
        c[k] = 2.0 * acc / (double)n;
    }
    c[0] *= 0.5;
    return FR_OK;
}

extern "C" int fr_cheb_ps_params(int32_t degree, int32_t *d1, int32_t *d2) {
    if (degree < 1 || !d1 || !d2) return fr_fail(FR_EINVAL, "fr_cheb_ps_params: bad arguments");
    int best = INT_MAX;
    for (int a = 2; a <= degree + 1; ++a) {
        int b = 1;
        while ((long long)a << (b - 1) < degree) ++b;
        if (a + b < best) {
            best = a + b;
            *d1 = a;
            *d2 = b;
        }
    }
    return FR_OK;
}

extern "C" int fr_stream_pool_size(int32_t units, double free_bytes, double ct_bytes) {
    if (units <= 0 || ct_bytes <= 0) return fr_fail(FR_EINVAL, "fr_stream_pool_size: bad arguments");
    long long s = std::min<long long>(units / 4, (long long)std::floor(0.2 * free_bytes / (40.0 * ct_bytes)));
    s = std::min<long long>(s, 32);
    return (int)std::max<long long>(s, 2);
}

extern "C" int fr_bsgs_rotation_set(int32_t ell, int32_t n1, int32_t *out, int32_t cap) {
    if (ell <= 0 || n1 <= 0 || n1 > ell) return fr_fail(FR_EINVAL, "fr_bsgs_rotation_set: bad arguments");
    const int n2 = (ell + n1 - 1) / n1;
    int n = 0;
    for (int i = 1; i < n1; ++i) {
        if (out && n < cap) out[n] = i;
        ++n;
    }
    for (int j = 1; j < n2; ++j) {
        if (out && n < cap) out[n] = j * n1;
        ++n;
    }
    return n;
}
