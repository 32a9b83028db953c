// kernels_rns.hip -- residue-number-system kernels of the hot path (gfx950):
// pointwise ring arithmetic, the Galois automorphism, hybrid key switching
// (ModUp fast base conversion, key inner product, ModDown), rescale and the
// fused plaintext-diagonal multiply-accumulate of the BSGS inner sums.
//
// All kernels are HBM-streaming: one thread per (limb, coefficient) word,
// 256 threads per workgroup, limbs on grid.y, polynomials on grid.z.
#include <algorithm>

#include "fr_core.h"

namespace {

constexpr int kT = 256;
constexpr int kMaxDigit = 8;  // alpha <= 8 (checked at context creation)
constexpr int kTargetsPerThread = 8;  // ModUp conversions: target limbs per thread
constexpr int kFbcTargets = 8;  // ModDown conversions: target limbs per thread

// Exact sum of at most 16 products y w with y, w < 2^60 (residues and table
// constants of primes below 2^60).  With 30-bit halves y = y0 + y1 2^30 and
// w = w0 + w1 2^30, each of the four partial sums (y0 w0, y0 w1, y1 w0,
// y1 w1) stays below 2^64 (terms below 2^60, plus a start value below 2^60
// in the first), so a term takes four 32 x 32 -> 64-bit multiply-adds and no
// carry handling; the 128-bit total is formed once.
__device__ __forceinline__ void split30(u64 y, u32 &y0, u32 &y1) {
    y0 = (u32)y & 0x3fffffffu;
    y1 = (u32)(y >> 30);
}
struct Dot30 {
    u64 a, b1 = 0, b2 = 0, c = 0;
    __device__ __forceinline__ explicit Dot30(u64 start = 0) : a(start) {}
    __device__ __forceinline__ void add(u32 y0, u32 y1, u32 w0, u32 w1) {
        a += (u64)y0 * w0;
        b1 += (u64)y0 * w1;
        b2 += (u64)y1 * w0;
        c += (u64)y1 * w1;
    }
    __device__ __forceinline__ void add(u32 y0, u32 y1, u64 w) {
        u32 w0, w1;
        split30(w, w0, w1);
        add(y0, y1, w0, w1);
    }
    __device__ __forceinline__ unsigned __int128 total() const {
        return (unsigned __int128)a + (((unsigned __int128)b1 + b2) << 30) + ((unsigned __int128)c << 60);
    }
    // (total) 2^-64 mod q
    __device__ __forceinline__ u64 redc(const ModConst &m) const {
        const unsigned __int128 s = total();
        return redc_any((u64)s, (u64)(s >> 64), m);
    }
};

// ModDown's overflow count e = round(X / P) for X = sum_j y_j Phat_j in
// [0, nP P) (y_j < p_j, Phat_j = P / p_j), i.e. the e that makes X - e P the
// centered residue of the input mod P.  X / P = sum_j y_j / p_j is summed in
// FP64 (fixed order, no contraction): |error| < 2^-46 for nP <= 8 terms below
// 1 each, so rint() is exact unless the sum lies within 2^-40 of a
// half-integer.  There the decision is taken in integers: with k = floor(s),
// e = k + 1 exactly when 2 X > (2k + 1) P (P is odd, so the two never tie),
// compared in kPW-word arithmetic against the tables Phat_j and P.
constexpr int kPW = kMaxDigit + 1;  // 64-bit words of the multiword integers
static_assert(kPW == kPbigWords && kMaxDigit + 1 == kPbigRows, "multiword table shape");
__device__ __forceinline__ u64 overflow_exact(const u64 (&y)[kMaxDigit], int nP, double s, const u64 *pbig) {
    u64 X[kPW];
#pragma unroll
    for (int w = 0; w < kPW; ++w) X[w] = 0;
#pragma unroll
    for (int j = 0; j < kMaxDigit; ++j)
        if (j < nP) {
            u64 carry = 0;
#pragma unroll
            for (int w = 0; w < kPW; ++w) {
                const u64 ph = pbig[j * kPW + w];
                u64 lo = ph * y[j], hi = mulhi64(ph, y[j]);
                lo += X[w];
                hi += lo < X[w] ? 1u : 0u;
                lo += carry;
                hi += lo < carry ? 1u : 0u;
                X[w] = lo;
                carry = hi;
            }
        }
    const u64 k = (u64)floor(s), m = 2 * k + 1;
    const u64 *P = pbig + kMaxDigit * kPW;
    u64 ycarry = 0, prev = 0, borrow = 0;
#pragma unroll
    for (int w = 0; w < kPW; ++w) {
        const u64 x2 = (X[w] << 1) | (prev >> 63);  // word w of 2 X
        prev = X[w];
        u64 yl = P[w] * m;                           // word w of (2k + 1) P
        const u64 yh = mulhi64(P[w], m);
        yl += ycarry;
        ycarry = yh + (yl < ycarry ? 1u : 0u);
        const u64 d = x2 - yl;                       // 2 X - (2k + 1) P, with borrow
        const u64 b1 = x2 < yl ? 1u : 0u;
        const u64 b2 = d < borrow ? 1u : 0u;
        borrow = b1 | b2;
    }
    return borrow ? k : k + 1;
}
__device__ __forceinline__ u64 overflow_round(const u64 (&y)[kMaxDigit], int nP, double s, const u64 *pbig) {
    const double f = s - floor(s);
    if (fabs(f - 0.5) < 0x1p-40) return overflow_exact(y, nP, s, pbig);
    return (u64)rint(s);
}

// Batch item and tile of a block when every tile is processed for `batch`
// items.  Workgroups are placed on the 8 XCDs round-robin by linear id, so
// with ntiles a multiple of 8 the `batch` blocks of one tile are consecutive
// on one XCD and share its L2 (one HBM read of the shared operand); other
// shapes fall back to items varying fastest.
__device__ __forceinline__ void item_tile(int b, int batch, int ntiles, int &item, int &tile) {
    if ((ntiles & 7) == 0) {
        const int s = b >> 3;
        item = s % batch;
        tile = (s / batch) * 8 + (b & 7);
    } else {
        item = b % batch;
        tile = b / batch;
    }
}

struct LimbConsts {
    u64 v[FR_MAXMOD];
    u64 sh[FR_MAXMOD];
};

__global__ __launch_bounds__(kT) void k_add(u64 *out, const u64 *a, const u64 *b, int N, size_t so,
                                            size_t sa, size_t sb, const ModConst *mods, int subtract) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z;
    const u64 q = mods[i].q;
    const size_t w = (size_t)i * N + k;
    const u64 x = a[p * sa + w], y = b[p * sb + w];
    out[p * so + w] = subtract ? subq(x, y, q) : addq(x, y, q);
}

__global__ __launch_bounds__(kT) void k_mul_const(u64 *out, const u64 *a, LimbConsts kc, int N, size_t so,
                                                  size_t sa, const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z;
    const size_t w = (size_t)i * N + k;
    out[p * so + w] = shoup(a[p * sa + w], kc.v[i], kc.sh[i], mods[i].q);
}

__global__ __launch_bounds__(kT) void k_add_const(u64 *out, const u64 *a, LimbConsts kc, int N,
                                                  const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const size_t w = (size_t)i * N + k;
    out[w] = addq(a[w], kc.v[i], mods[i].q);
}

__global__ __launch_bounds__(kT) void k_mul_pt(u64 *out, const u64 *a, const u64 *b, int N, size_t so,
                                               size_t sa, const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z;
    const size_t w = (size_t)i * N + k;
    out[p * so + w] = mulmod(a[p * sa + w], b[w], mods[i]);
}

__global__ __launch_bounds__(kT) void k_tensor(u64 *d0, u64 *d1, u64 *d2, const u64 *a0, const u64 *a1,
                                               const u64 *b0, const u64 *b1, int N, const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const ModConst m = mods[i];
    const size_t w = (size_t)i * N + k;
    const u64 x0 = a0[w], x1 = a1[w], y0 = b0[w], y1 = b1[w];
    d0[w] = mulmod(x0, y0, m);
    d1[w] = addq(mulmod(x0, y1, m), mulmod(x1, y0, m), m.q);
    d2[w] = mulmod(x1, y1, m);
}

__global__ __launch_bounds__(kT) void k_automorph(u64 *out, const u64 *in, u64 g, int N, int logN, size_t so,
                                                  size_t si, const ModConst *mods, int accumulate) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z;
    const size_t w = (size_t)i * N + k;
    const u64 v = in[p * si + (size_t)i * N + auto_src((u32)k, g, logN)];
    out[p * so + w] = accumulate ? addq(out[p * so + w], v, mods[i].q) : v;
}

__global__ __launch_bounds__(kT) void k_mont_scale(u64 *data, int N, size_t ps, LimbMap map,
                                                   const ModConst *mods, int to_mont) {
    const int k = blockIdx.x * kT + threadIdx.x;
    const int s = map.storage(blockIdx.y);
    const ModConst m = mods[map.modidx(s)];
    u64 &x = data[blockIdx.z * ps + (size_t)s * N + k];
    x = to_mont ? shoup(x, m.r64, m.r64_sh, m.q) : redc(x, 0, m);
}

// ModUp of digit [lo, lo+nd): x coefficient form [level+1][N]; D[nE][N].
// y_d = [x_{lo+d} * Dhat_d^-1]_{q_{lo+d}} (canonical), then for every
// extended position e outside the digit: D[e] = sum_d y_d * [Dhat_d]_{r_e} mod r_e
// (table entries Montgomery-scaled: one reduction of the 128-bit sum).
// ND > 0: compiled for exactly ND limbs in the digit; ND = 0: any size
template <int ND>
__global__ __launch_bounds__(kT) void k_modup(u64 *__restrict__ D, const u64 *__restrict__ x, int N, int lo, int nd_rt,
                                              int nE, int level, int pbase, const u64 *__restrict__ tab,
                                              const ModConst *__restrict__ mods, size_t sd, size_t sx,
                                              const u64 *__restrict__ own, size_t so) {
    const int nd = ND ? ND : nd_rt;
    const int k = blockIdx.x * kT + threadIdx.x;
    D += blockIdx.z * sd;
    x += blockIdx.z * sx;
    if (own && blockIdx.y == 0) {  // the digit's own limbs, evaluation form as given
        own += blockIdx.z * so;
#pragma unroll
        for (int d = 0; d < kMaxDigit; ++d)
            if (d < nd) D[(size_t)(lo + d) * N + k] = own[(size_t)(lo + d) * N + k];
    }
    const u64 *dinv = tab, *dinv_sh = tab + nd, *dhat = tab + 2 * nd;
    u32 y0[kMaxDigit], y1[kMaxDigit];
#pragma unroll
    for (int d = 0; d < kMaxDigit; ++d)
        if (d < nd) split30(shoup(x[(size_t)(lo + d) * N + k], dinv[d], dinv_sh[d], mods[lo + d].q), y0[d], y1[d]);
    const int ntarget = nE - nd;
    const int t0 = blockIdx.y * kTargetsPerThread, t1 = min(ntarget, t0 + kTargetsPerThread);
    for (int te = t0; te < t1; ++te) {
        const int e = te < lo ? te : te + nd;
        const int gm = e <= level ? e : pbase + (e - level - 1);
        Dot30 acc;
#pragma unroll
        for (int d = 0; d < kMaxDigit; ++d)
            if (d < nd) acc.add(y0[d], y1[d], dhat[(size_t)e * nd + d]);
        D[(size_t)e * N + k] = acc.redc(mods[gm]);
    }
}

// ModUp of every digit in one launch: grid.z = item * ndig + t.  Digit t of
// item b fills D[b][t][e] for all e < nE: the converted value outside the
// digit (as k_modup) and, inside it, the digit's own coefficients x_e, so
// that one forward transform over all nE limbs gives the extended digit (the
// transform of x_e is the input limb's evaluation form word for word).
struct ModupTabs {
    const u64 *tab[kMaxDigit];
};
template <int ND>
__device__ __forceinline__ void modup_all_body(u64 *D, const u64 *x, int N, int tfirst, int nt, int alpha, int nE,
                                               int level, int pbase, const ModupTabs &mt, const ModConst *mods,
                                               size_t sd, size_t sx, const u64 *own, size_t so) {
    const int k = blockIdx.x * kT + threadIdx.x;
    const int t = tfirst + blockIdx.z % nt, b = blockIdx.z / nt;
    const int lo = t * alpha, nd = ND ? ND : min(alpha, level + 1 - lo);
    D += b * sd + (size_t)t * nE * N;
    x += b * sx;
    if (own) own += b * so;
    const u64 *tab = mt.tab[t - tfirst];
    const u64 *dinv = tab, *dinv_sh = tab + nd, *dhat = tab + 2 * nd;
    u32 y0[kMaxDigit], y1[kMaxDigit];
#pragma unroll
    for (int d = 0; d < kMaxDigit; ++d)
        if (d < nd) {
            const u64 xv = x[(size_t)(lo + d) * N + k];
            if (blockIdx.y == 0) D[(size_t)(lo + d) * N + k] = own ? own[(size_t)(lo + d) * N + k] : xv;
            split30(shoup(xv, dinv[d], dinv_sh[d], mods[lo + d].q), y0[d], y1[d]);
        }
    const int ntarget = nE - nd;
    const int t0 = blockIdx.y * kTargetsPerThread, t1 = min(ntarget, t0 + kTargetsPerThread);
    for (int te = t0; te < t1; ++te) {
        const int e = te < lo ? te : te + nd;
        const int gm = e <= level ? e : pbase + (e - level - 1);
        Dot30 acc;
#pragma unroll
        for (int d = 0; d < kMaxDigit; ++d)
            if (d < nd) acc.add(y0[d], y1[d], dhat[(size_t)e * nd + d]);
        D[(size_t)e * N + k] = acc.redc(mods[gm]);
    }
}

// ALPHA > 0: digits of ALPHA limbs take the body compiled for that size (a
// shorter last digit takes the general one)
template <int ALPHA>
__global__ __launch_bounds__(kT) void k_modup_all(u64 *__restrict__ D, const u64 *__restrict__ x, int N, int tfirst,
                                                  int nt, int alpha, int nE, int level, int pbase, ModupTabs mt,
                                                  const ModConst *__restrict__ mods, size_t sd, size_t sx,
                                                  const u64 *__restrict__ own, size_t so) {
    const int t = tfirst + blockIdx.z % nt;
    if (ALPHA && min(alpha, level + 1 - t * alpha) == ALPHA)
        modup_all_body<ALPHA>(D, x, N, tfirst, nt, alpha, nE, level, pbase, mt, mods, sd, sx, own, so);
    else
        modup_all_body<0>(D, x, N, tfirst, nt, alpha, nE, level, pbase, mt, mods, sd, sx, own, so);
}

// U{0,1}[e][p] (+)= sum_t D_t[e][src(p)] * ksk_t{b,a}[gm(e)][p]; keys are
// Montgomery-scaled so one reduction yields the canonical sum.
// fold (relinearisation): the top limb of U becomes d_l + P^-1 U_l (d an item
// of fold_sd words, [2][level+1][N]); U_l is read by nothing else afterwards
// one key word: a 64-bit limb, or a packed limb's low word and high byte
template <bool PK>
__device__ __forceinline__ u64 key_word(const unsigned char *limb, int p, int N) {
    if (PK) return (u64)reinterpret_cast<const u32 *>(limb)[p] | ((u64)limb[4 * (size_t)N + p] << 32);
    return reinterpret_cast<const u64 *>(limb)[p];
}

// ND > 0: compiled for exactly ND digits, every word of the thread in flight
// before the sums (ND = 0: any count, one digit at a time).  PK: the key limb
// is packed (5 bytes per word).
template <int ND, bool PK>
__device__ __forceinline__ void ks_inner_body(u64 *U0, u64 *U1, const u64 *D, const unsigned char *kl0,
                                              size_t kblock, u32 src, int p, int e, int N, int nE, int level,
                                              int ndig, const ModConst &m, int accumulate, int item,
                                              const u64 *fold_d, size_t fold_sd, u64 pinv_top, u64 pinv_top_sh,
                                              const u64 *rot_c0, size_t c0_sd, const u64 *pmont) {
    // key limb of digit t, part ab (0: b, 1: a)
    auto kw = [&](int t, int ab) { return key_word<PK>(kl0 + (size_t)(t * 2 + ab) * kblock, p, N); };
    Dot30 s0, s1;
    if constexpr (ND > 0) {
        u64 d[ND], kb[ND], ka[ND];
#pragma unroll
        for (int t = 0; t < ND; ++t) {
            d[t] = D[((size_t)t * nE + e) * N + src];
            kb[t] = kw(t, 0);
            ka[t] = kw(t, 1);
        }
        const u64 c0 = (rot_c0 && e <= level) ? rot_c0[item * c0_sd + (size_t)e * N + src] : 0;
#pragma unroll
        for (int t = 0; t < ND; ++t) {
            u32 d0, d1;
            split30(d[t], d0, d1);
            s0.add(d0, d1, kb[t]);
            s1.add(d0, d1, ka[t]);
        }
        if (rot_c0 && e <= level) {
            u32 c00, c01;
            split30(c0, c00, c01);
            s0.add(c00, c01, pmont[e]);
        }
    } else {
        for (int t = 0; t < ndig; ++t) {
            u32 d0, d1;
            split30(D[((size_t)t * nE + e) * N + src], d0, d1);
            s0.add(d0, d1, kw(t, 0));
            s1.add(d0, d1, kw(t, 1));
        }
        if (rot_c0 && e <= level) {
            u32 c00, c01;
            split30(rot_c0[item * c0_sd + (size_t)e * N + src], c00, c01);
            s0.add(c00, c01, pmont[e]);
        }
    }
    u64 u0 = s0.redc(m), u1 = s1.redc(m);
    const size_t w = (size_t)e * N + p;
    if (accumulate) {
        u0 = addq(u0, U0[w], m.q);
        u1 = addq(u1, U1[w], m.q);
    }
    if (fold_d && e == level) {
        const u64 *d = fold_d + item * fold_sd + w;
        u0 = addq(d[0], shoup(u0, pinv_top, pinv_top_sh, m.q), m.q);
        u1 = addq(d[(size_t)(level + 1) * N], shoup(u1, pinv_top, pinv_top_sh, m.q), m.q);
    }
    U0[w] = u0;
    U1[w] = u1;
}

template <int ND>
__global__ __launch_bounds__(kT) void k_ks_inner(u64 *__restrict__ U0, u64 *__restrict__ U1, const u64 *__restrict__ D, const unsigned char *__restrict__ ksk,
                                                 KeyLayout kl, u64 g, int N, int logN, int nE, int level, int pbase,
                                                 int ndig, const ModConst *__restrict__ mods, int accumulate, size_t sd, size_t su,
                                                 int batch, const u64 *__restrict__ fold_d, size_t fold_sd, u64 pinv_top,
                                                 u64 pinv_top_sh, const u64 *__restrict__ rot_c0, size_t c0_sd,
                                                 const u64 *__restrict__ pmont) {
    int item, tile;
    item_tile(blockIdx.x, batch, N / kT, item, tile);
    const int p = tile * kT + threadIdx.x, e = blockIdx.y;
    D += item * sd;
    U0 += item * su;
    U1 += item * su;
    const int gm = e <= level ? e : pbase + (e - level - 1);
    const ModConst m = mods[gm];
    const u32 src = g == 1 ? (u32)p : auto_src((u32)p, g, logN);
    const unsigned char *kl0 = ksk + kl.off[gm];
    if (kl.packed[gm])
        ks_inner_body<ND, true>(U0, U1, D, kl0, kl.block, src, p, e, N, nE, level, ndig, m, accumulate, item, fold_d,
                                fold_sd, pinv_top, pinv_top_sh, rot_c0, c0_sd, pmont);
    else
        ks_inner_body<ND, false>(U0, U1, D, kl0, kl.block, src, p, e, N, nE, level, ndig, m, accumulate, item, fold_d,
                                 fold_sd, pinv_top, pinv_top_sh, rot_c0, c0_sd, pmont);
}

// Key inner products of several hoisted rotations of one ModUp digit set,
// each output over Q_l U P with P sigma_g(c0) folded in (the baby steps of
// the hoisted product): for rotation b with Galois element g_b,
//   U0_b[e][p] = sum_t D_t[e][s] * ksk_{b,t,b}[gm(e)][p] + P c0[e][s] (e <= level),
//   U1_b[e][p] = sum_t D_t[e][s] * ksk_{b,t,a}[gm(e)][p],
// with s = auto_src(p, g_b).  A thread owns one source word s: it reads the
// digit words D_t[e][s] and c0[e][s] once and, for each rotation, writes
// output p = auto_src(s, g_b^-1) (the automorphism maps every aligned block
// of 64 words onto an aligned block of 64 words, so a wave's keys and
// outputs still fill whole cache lines).  The digit set and c0 are read
// once for all the rotations instead of once per rotation.  The outputs
// (31 baby steps of 20 MiB at N = 2^16, more than the last-level cache
// holds) are written with non-temporal stores, so that their write-backs
// do not fall into the MAC that reads them next.
constexpr int kMultiRot = 32;
struct MultiKeys {
    const unsigned char *ksk[kMultiRot];
    u64 ginv[kMultiRot];
};
// 16 zero bytes: the source of the global-to-LDS loads of a stage's padding
// (and, in the MAC, of diagonals past ell or nj)
__device__ __align__(16) uint4 g_zero16 = {0u, 0u, 0u, 0u};

// cache-policy operand of a global-to-LDS load: non-temporal.  A one-query
// MAC streams its words once, and they should not displace what the caches
// hold for the kernels around it; with several queries per launch the
// blocks of one tile share it through the L2, and the default policy is
// kept (measured: 2.84 -> 2.79 ms for the one-query product, 4.00 -> 3.96
// ms per query batched when the batched launch keeps the default).
constexpr int kCachePolicyNT = 2;

// A block's 256 sources s map, for every rotation, onto one aligned block
// of 256 outputs p (P0 ... P0 + 255).  So the key words a rotation needs are
// whole 256-word slices of its 2 ND key limbs: they are copied from HBM into
// one of two LDS stages, one rotation ahead, by wave-wide 16-byte
// global-to-LDS loads (lane l of a load lands at byte 16 l of its 1 KiB
// chunk), and each thread reads its words at p - P0 from there.  A stage
// holds the slices' low words (1 KiB each) then their high bytes (256 B
// each) for packed limbs, or the 2 KiB slices of 64-bit limbs.
template <int ND, bool PK>
constexpr int ks_multi_stage_bytes() {
    return ((2 * ND * (PK ? 1280 : 2048) + 1023) / 1024) * 1024;
}
template <int ND, bool PK>
__device__ __forceinline__ void ks_multi_body(u64 *U, size_t ub, const u64 *D, const MultiKeys &mk, int nrot,
                                              size_t kblock, unsigned koff, u32 s0w, int e, int N, int logN, int nE,
                                              int level, const ModConst &m, const u64 *c0, const u64 *pmont,
                                              unsigned char *lds) {
    constexpr int NL = 2 * ND;                           // key limbs of a rotation: digit t, part b / a
    constexpr int LOP = PK ? 64 : 128;                   // 16-byte pieces of a limb's slice (low words)
    constexpr int TOT = NL * LOP + (PK ? NL * 16 : 0);  // pieces of a stage
    constexpr int NCH = (TOT + 63) / 64, STG = NCH * 1024;
    static_assert(STG == ks_multi_stage_bytes<ND, PK>(), "stage stride");
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const u32 s = s0w + t;
    u32 d0[ND], d1[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) split30(D[((size_t)i * nE + e) * N + s], d0[i], d1[i]);
    u32 c00 = 0, c01 = 0;
    const bool has_c0 = e <= level;
    if (has_c0) split30(c0[(size_t)e * N + s], c00, c01);
    const u64 pm = has_c0 ? pmont[e] : 0;
    auto dma = [&](int b, int st) {
        const u32 P0 = auto_src(s0w, mk.ginv[b], logN) & ~255u;
        const unsigned char *kl0 = mk.ksk[b] + koff;
        unsigned char *dst = lds + st * STG;
#pragma unroll
        for (int c = wv; c < NCH; c += kT / 64) {
            const int i = c * 64 + lane;
            const void *src = &g_zero16;
            if (i < NL * LOP) {
                const int li = i / LOP, w = i - li * LOP;
                src = kl0 + (size_t)li * kblock + (PK ? 4 : 8) * (size_t)P0 + 16 * w;
            } else if (i < TOT) {
                const int j = i - NL * LOP, li = j >> 4;
                src = kl0 + (size_t)li * kblock + 4 * (size_t)N + P0 + 16 * (j & 15);
            }
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(dst + c * 1024), 16, 0,
                                             0);
        }
    };
    dma(0, 0);
    for (int b = 0; b < nrot; ++b) {
        __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0): this wave's loads of stage b
        __syncthreads();                      // every wave's, and every wave done with stage b - 1
        if (b + 1 < nrot) dma(b + 1, (b + 1) & 1);
        const u32 p = auto_src(s, mk.ginv[b], logN), r = p & 255u;
        const unsigned char *st = lds + (b & 1) * STG;
        auto kw = [&](int li) -> u64 {
            if (PK)
                return (u64)reinterpret_cast<const u32 *>(st + li * 1024)[r] |
                       ((u64)st[NL * 1024 + li * 256 + r] << 32);
            return reinterpret_cast<const u64 *>(st + li * 2048)[r];
        };
        Dot30 s0, s1;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            s0.add(d0[i], d1[i], kw(2 * i));
            s1.add(d0[i], d1[i], kw(2 * i + 1));
        }
        if (has_c0) s0.add(c00, c01, pm);
        u64 *Ub = U + b * ub + (size_t)e * N + p;
        __builtin_nontemporal_store(s0.redc(m), Ub);
        __builtin_nontemporal_store(s1.redc(m), Ub + (size_t)nE * N);
    }
}

template <int ND>
__global__ __launch_bounds__(kT) void k_ks_inner_multi(u64 *__restrict__ U, size_t ub, const u64 *__restrict__ D, MultiKeys mk, int nrot,
                                                       KeyLayout kl, int N, int logN, int nE, int level, int pbase,
                                                       const ModConst *__restrict__ mods, size_t sd, size_t su, int batch,
                                                       const u64 *__restrict__ c0, size_t c0_sd, const u64 *__restrict__ pmont) {
    __shared__ __align__(16) unsigned char lds[2 * ks_multi_stage_bytes<ND, false>()];
    int item, tile;
    item_tile(blockIdx.x, batch, N / kT, item, tile);
    const u32 s0w = tile * kT;
    const int e = blockIdx.y;
    const int gm = e <= level ? e : pbase + (e - level - 1);
    const ModConst m = mods[gm];
    D += item * sd;
    U += item * su;
    c0 += item * c0_sd;
    if (kl.packed[gm])
        ks_multi_body<ND, true>(U, ub, D, mk, nrot, kl.block, kl.off[gm], s0w, e, N, logN, nE, level, m, c0, pmont,
                                lds);
    else
        ks_multi_body<ND, false>(U, ub, D, mk, nrot, kl.block, kl.off[gm], s0w, e, N, logN, nE, level, m, c0, pmont,
                                 lds);
}

// Summed tensor products of ciphertext pairs (encrypted-database product):
// t01 (+)= (sum a0 b0, sum a0 b1 + a1 b0), t2 (+)= sum a1 b1 over up to
// kPairs pairs per launch, each sum a 128-bit lazy accumulation of at most
// 2 kPairs = 64 products below 2^122, reduced once.
constexpr int kPairs = 32;
struct PairPtrs {
    const u64 *a[kPairs];
    const u64 *b[kPairs];
};
__global__ __launch_bounds__(kT) void k_tensor_sum(u64 *t01, u64 *t2, PairPtrs pp, int np, int nl, int N,
                                                   const ModConst *mods, int accumulate) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const ModConst m = mods[i];
    const size_t lw = (size_t)nl * N, w = (size_t)i * N + k;
    u64 l0 = 0, h0 = 0, l1 = 0, h1 = 0, l2 = 0, h2 = 0;
    for (int p = 0; p < np; ++p) {
        const u64 x0 = pp.a[p][w], x1 = pp.a[p][lw + w], y0 = pp.b[p][w], y1 = pp.b[p][lw + w];
        mac128(l0, h0, x0, y0);
        mac128(l1, h1, x0, y1);
        mac128(l1, h1, x1, y0);
        mac128(l2, h2, x1, y1);
    }
    u64 r0 = reduce128(l0, h0, m), r1 = reduce128(l1, h1, m), r2 = reduce128(l2, h2, m);
    if (accumulate) {
        r0 = addq(r0, t01[w], m.q);
        r1 = addq(r1, t01[lw + w], m.q);
        r2 = addq(r2, t2[w], m.q);
    }
    t01[w] = r0;
    t01[lw + w] = r1;
    t2[w] = r2;
}

// Sum of the key inner products of several rotations (the giant steps of
// one BSGS product, accumulated in the extended basis before one ModDown):
// U{0,1}[e][p] (+)= sum_j sum_t D_{j,t}[e][auto_src(p, g_j)] * ksk_{j,t}[gm(e)][p].
// The 128-bit lazy sum holds nj * ndig <= 64 products below 2^122.
constexpr int kGiant = 16;
struct GiantKeys {
    const unsigned char *ksk[kGiant];
    u64 g[kGiant];
};
template <int ND, bool PK>
__device__ __forceinline__ void ks_inner_sum_body(u64 *U0, u64 *U1, const u64 *D, const GiantKeys &gk, int nj,
                                                  size_t sdj, unsigned koff, size_t kblock, int p, int e, int N,
                                                  int logN, int nE, int ndig, const ModConst &m, int accumulate) {
    // exact sums of each giant step's digits (Dot30), added up in 128 bits
    unsigned __int128 t0 = 0, t1 = 0;
    for (int jj = 0; jj < nj; ++jj) {
        const u32 src = auto_src((u32)p, gk.g[jj], logN);
        const u64 *Dj = D + jj * sdj;
        const unsigned char *kl0 = gk.ksk[jj] + koff;
        auto kw = [&](int t, int ab) { return key_word<PK>(kl0 + (size_t)(t * 2 + ab) * kblock, p, N); };
        Dot30 s0, s1;
        if constexpr (ND > 0) {
            u64 d[ND], kb[ND], ka[ND];
#pragma unroll
            for (int t = 0; t < ND; ++t) {
                d[t] = Dj[((size_t)t * nE + e) * N + src];
                kb[t] = kw(t, 0);
                ka[t] = kw(t, 1);
            }
#pragma unroll
            for (int t = 0; t < ND; ++t) {
                u32 d0, d1;
                split30(d[t], d0, d1);
                s0.add(d0, d1, kb[t]);
                s1.add(d0, d1, ka[t]);
            }
        } else {
            for (int t = 0; t < ndig; ++t) {
                u32 d0, d1;
                split30(Dj[((size_t)t * nE + e) * N + src], d0, d1);
                s0.add(d0, d1, kw(t, 0));
                s1.add(d0, d1, kw(t, 1));
            }
        }
        t0 += s0.total();
        t1 += s1.total();
    }
    u64 u0 = redc_any((u64)t0, (u64)(t0 >> 64), m), u1 = redc_any((u64)t1, (u64)(t1 >> 64), m);
    const size_t w = (size_t)e * N + p;
    if (accumulate) {
        u0 = addq(u0, U0[w], m.q);
        u1 = addq(u1, U1[w], m.q);
    }
    U0[w] = u0;
    U1[w] = u1;
}

template <int ND>
__global__ __launch_bounds__(kT) void k_ks_inner_sum(u64 *__restrict__ U0, u64 *__restrict__ U1, const u64 *__restrict__ D, GiantKeys gk, KeyLayout kl,
                                                     int nj, size_t sdj, int N, int logN, int nE, int level,
                                                     int pbase, int ndig, const ModConst *__restrict__ mods, int accumulate,
                                                     size_t sd, size_t su, int batch) {
    int item, tile;
    item_tile(blockIdx.x, batch, N / kT, item, tile);
    const int p = tile * kT + threadIdx.x, e = blockIdx.y;
    D += item * sd;
    U0 += item * su;
    U1 += item * su;
    const int gm = e <= level ? e : pbase + (e - level - 1);
    const ModConst m = mods[gm];
    if (kl.packed[gm])
        ks_inner_sum_body<ND, true>(U0, U1, D, gk, nj, sdj, kl.off[gm], kl.block, p, e, N, logN, nE, ndig, m,
                                    accumulate);
    else
        ks_inner_sum_body<ND, false>(U0, U1, D, gk, nj, sdj, kl.off[gm], kl.block, p, e, N, logN, nE, ndig, m,
                                     accumulate);
}

// The same sums with the key words staged through LDS (ND = 1..3): a
// block's 256 outputs P0 .. P0+255 read, for every giant step, whole
// 256-word slices of its 2 ND key limbs; they are copied from HBM into one
// of two LDS stages one giant step ahead by wave-wide 16-byte global-to-LDS
// loads (the layout of the baby steps' kernel), and the digit words of the
// next giant step are loaded per lane meanwhile.
template <int ND, bool PK>
__device__ __forceinline__ void ks_sum_lds_body(u64 *U0, u64 *U1, const u64 *D, const GiantKeys &gk, int nj,
                                                size_t sdj, unsigned koff, size_t kblock, u32 P0, int e, int N,
                                                int logN, int nE, const ModConst &m, int accumulate, bool nt,
                                                unsigned char *lds) {
    constexpr int NL = 2 * ND;
    constexpr int LOP = PK ? 64 : 128;
    constexpr int TOT = NL * LOP + (PK ? NL * 16 : 0);
    constexpr int NCH = (TOT + 63) / 64, STG = NCH * 1024;
    static_assert(STG == ks_multi_stage_bytes<ND, PK>(), "stage stride");
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const u32 p = P0 + t;
    auto dma = [&](int jj, int st) {
        const unsigned char *kl0 = gk.ksk[jj] + koff;
        unsigned char *dst = lds + st * STG;
#pragma unroll
        for (int c = wv; c < NCH; c += kT / 64) {
            const int i = c * 64 + lane;
            const void *src = &g_zero16;
            if (i < NL * LOP) {
                const int li = i / LOP, w = i - li * LOP;
                src = kl0 + (size_t)li * kblock + (PK ? 4 : 8) * (size_t)P0 + 16 * w;
            } else if (i < TOT) {
                const int j = i - NL * LOP, li = j >> 4;
                src = kl0 + (size_t)li * kblock + 4 * (size_t)N + P0 + 16 * (j & 15);
            }
            auto *d = (__attribute__((address_space(3))) void *)(dst + c * 1024);
            if (nt)
                __builtin_amdgcn_global_load_lds(src, d, 16, 0, kCachePolicyNT);
            else
                __builtin_amdgcn_global_load_lds(src, d, 16, 0, 0);
        }
    };
    auto digits = [&](int jj, u64 (&d)[ND]) {
        const u32 src = auto_src(p, gk.g[jj], logN);
        const u64 *Dj = D + jj * sdj;
#pragma unroll
        for (int i = 0; i < ND; ++i) d[i] = Dj[((size_t)i * nE + e) * N + src];
    };
    unsigned __int128 t0 = 0, t1 = 0;
    u64 d[ND];
    dma(0, 0);
    digits(0, d);
    for (int jj = 0; jj < nj; ++jj) {
        __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0): this wave's stage jj and digit words
        __syncthreads();                      // every wave's, and every wave done with stage jj - 1
        u32 d0[ND], d1[ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) split30(d[i], d0[i], d1[i]);
        if (jj + 1 < nj) {
            dma(jj + 1, (jj + 1) & 1);
            digits(jj + 1, d);
        }
        const unsigned char *st = lds + (jj & 1) * STG;
        auto kw = [&](int li) -> u64 {
            if (PK)
                return (u64)reinterpret_cast<const u32 *>(st + li * 1024)[t] |
                       ((u64)st[NL * 1024 + li * 256 + t] << 32);
            return reinterpret_cast<const u64 *>(st + li * 2048)[t];
        };
        Dot30 s0, s1;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            s0.add(d0[i], d1[i], kw(2 * i));
            s1.add(d0[i], d1[i], kw(2 * i + 1));
        }
        t0 += s0.total();
        t1 += s1.total();
    }
    u64 u0 = redc_any((u64)t0, (u64)(t0 >> 64), m), u1 = redc_any((u64)t1, (u64)(t1 >> 64), m);
    const size_t w = (size_t)e * N + p;
    if (accumulate) {
        u0 = addq(u0, U0[w], m.q);
        u1 = addq(u1, U1[w], m.q);
    }
    U0[w] = u0;
    U1[w] = u1;
}

template <int ND>
__global__ __launch_bounds__(kT) void k_ks_inner_sum_lds(u64 *__restrict__ U0, u64 *__restrict__ U1,
                                                         const u64 *__restrict__ D, GiantKeys gk, KeyLayout kl, int nj,
                                                         size_t sdj, int N, int logN, int nE, int level, int pbase,
                                                         const ModConst *__restrict__ mods, int accumulate, size_t sd,
                                                         size_t su, int batch) {
    __shared__ __align__(16) unsigned char lds[2 * ks_multi_stage_bytes<ND, false>()];
    int item, tile;
    item_tile(blockIdx.x, batch, N / kT, item, tile);
    const int e = blockIdx.y;
    D += item * sd;
    U0 += item * su;
    U1 += item * su;
    const int gm = e <= level ? e : pbase + (e - level - 1);
    const ModConst m = mods[gm];
    const u32 P0 = tile * kT;
    if (kl.packed[gm])
        ks_sum_lds_body<ND, true>(U0, U1, D, gk, nj, sdj, kl.off[gm], kl.block, P0, e, N, logN, nE, m, accumulate,
                                  batch == 1, lds);
    else
        ks_sum_lds_body<ND, false>(U0, U1, D, gk, nj, sdj, kl.off[gm], kl.block, P0, e, N, logN, nE, m, accumulate,
                                   batch == 1, lds);
}

// k_ks_inner with the key words staged through LDS (ND = 1..3): one key
// serves every item of the batch (a relinearisation wave, a batch of
// rotations by one element), so a block takes one tile of 256 outputs for
// all items: the tile's 2 ND key slices are copied into LDS once by
// wave-wide 16-byte global-to-LDS loads, then the items' sums follow, with
// the same epilogue (accumulation, fold, c0 term) as k_ks_inner.
template <int ND, bool PK>
__device__ __forceinline__ void ks_inner_lds_body(u64 *U0, u64 *U1, const u64 *D, const unsigned char *kl0,
                                                  size_t kblock, u64 g, u32 P0, int e, int N, int logN, int nE,
                                                  int level, const ModConst &m, int accumulate, int batch, size_t sd,
                                                  size_t su, const u64 *fold_d, size_t fold_sd, u64 pinv_top,
                                                  u64 pinv_top_sh, const u64 *rot_c0, size_t c0_sd, u64 pm,
                                                  unsigned char *lds) {
    constexpr int NL = 2 * ND;
    constexpr int LOP = PK ? 64 : 128;
    constexpr int TOT = NL * LOP + (PK ? NL * 16 : 0);
    constexpr int NCH = (TOT + 63) / 64;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const u32 p = P0 + t;
#pragma unroll
    for (int c = wv; c < NCH; c += kT / 64) {
        const int i = c * 64 + lane;
        const void *src = &g_zero16;
        if (i < NL * LOP) {
            const int li = i / LOP, w = i - li * LOP;
            src = kl0 + (size_t)li * kblock + (PK ? 4 : 8) * (size_t)P0 + 16 * w;
        } else if (i < TOT) {
            const int j = i - NL * LOP, li = j >> 4;
            src = kl0 + (size_t)li * kblock + 4 * (size_t)N + P0 + 16 * (j & 15);
        }
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(lds + c * 1024), 16, 0, 0);
    }
    const u32 src = g == 1 ? p : auto_src(p, g, logN);
    const bool has_c0 = rot_c0 && e <= level;
    auto load = [&](int item, u64 (&d)[ND], u64 &c0) {
#pragma unroll
        for (int i = 0; i < ND; ++i) d[i] = D[item * sd + ((size_t)i * nE + e) * N + src];
        c0 = has_c0 ? rot_c0[item * c0_sd + (size_t)e * N + src] : 0;
    };
    u64 d[ND], c0;
    load(0, d, c0);
    __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0): this wave's key pieces
    __syncthreads();                      // every wave's
    u64 kb[ND], ka[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
        auto kw = [&](int li) -> u64 {
            if (PK)
                return (u64)reinterpret_cast<const u32 *>(lds + li * 1024)[t] |
                       ((u64)lds[NL * 1024 + li * 256 + t] << 32);
            return reinterpret_cast<const u64 *>(lds + li * 2048)[t];
        };
        kb[i] = kw(2 * i);
        ka[i] = kw(2 * i + 1);
    }
    const size_t w = (size_t)e * N + p;
    for (int item = 0; item < batch; ++item) {
        u64 dn[ND], cn = 0;
        if (item + 1 < batch) load(item + 1, dn, cn);
        Dot30 s0, s1;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            u32 d0, d1;
            split30(d[i], d0, d1);
            s0.add(d0, d1, kb[i]);
            s1.add(d0, d1, ka[i]);
        }
        if (has_c0) {
            u32 c00, c01;
            split30(c0, c00, c01);
            s0.add(c00, c01, pm);
        }
        u64 u0 = s0.redc(m), u1 = s1.redc(m);
        u64 *O0 = U0 + item * su, *O1 = U1 + item * su;
        if (accumulate) {
            u0 = addq(u0, O0[w], m.q);
            u1 = addq(u1, O1[w], m.q);
        }
        if (fold_d && e == level) {
            const u64 *dd = fold_d + item * fold_sd + w;
            u0 = addq(dd[0], shoup(u0, pinv_top, pinv_top_sh, m.q), m.q);
            u1 = addq(dd[(size_t)(level + 1) * N], shoup(u1, pinv_top, pinv_top_sh, m.q), m.q);
        }
        O0[w] = u0;
        O1[w] = u1;
        if (item + 1 < batch) {
#pragma unroll
            for (int i = 0; i < ND; ++i) d[i] = dn[i];
            c0 = cn;
        }
    }
}

template <int ND>
__global__ __launch_bounds__(kT) void k_ks_inner_lds(u64 *__restrict__ U0, u64 *__restrict__ U1,
                                                     const u64 *__restrict__ D, const unsigned char *__restrict__ ksk,
                                                     KeyLayout kl, u64 g, int N, int logN, int nE, int level, int pbase,
                                                     const ModConst *__restrict__ mods, int accumulate, size_t sd,
                                                     size_t su, int batch, const u64 *__restrict__ fold_d,
                                                     size_t fold_sd, u64 pinv_top, u64 pinv_top_sh,
                                                     const u64 *__restrict__ rot_c0, size_t c0_sd,
                                                     const u64 *__restrict__ pmont) {
    __shared__ __align__(16) unsigned char lds[ks_multi_stage_bytes<ND, false>()];
    const int e = blockIdx.y;
    const int gm = e <= level ? e : pbase + (e - level - 1);
    const ModConst m = mods[gm];
    const u32 P0 = blockIdx.x * kT;
    const u64 pm = (rot_c0 && e <= level) ? pmont[e] : 0;
    if (kl.packed[gm])
        ks_inner_lds_body<ND, true>(U0, U1, D, ksk + kl.off[gm], kl.block, g, P0, e, N, logN, nE, level, m,
                                    accumulate, batch, sd, su, fold_d, fold_sd, pinv_top, pinv_top_sh, rot_c0, c0_sd,
                                    pm, lds);
    else
        ks_inner_lds_body<ND, false>(U0, U1, D, ksk + kl.off[gm], kl.block, g, P0, e, N, logN, nE, level, m,
                                     accumulate, batch, sd, su, fold_d, fold_sd, pinv_top, pinv_top_sh, rot_c0, c0_sd,
                                     pm, lds);
}

// out[b][i][k] (+)= sum_j in[b][j][i][auto_src(k, g_j)] (first polynomials of
// the giant steps; in items sij words apart per j and sib per b, out sob per
// b; limbs past `level` are the special primes, global index pbase + ...)
__global__ __launch_bounds__(kT) void k_automorph_sum(u64 *__restrict__ out, const u64 *__restrict__ in, GiantKeys gk, int nj, int N, int logN,
                                                      size_t sob, size_t sij, size_t sib, const ModConst *__restrict__ mods,
                                                      int level, int pbase, int accumulate) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, b = blockIdx.z;
    const u64 q = mods[i <= level ? i : pbase + (i - level - 1)].q;
    const u64 *ib = in + b * sib + (size_t)i * N;
    u64 acc = accumulate ? out[b * sob + (size_t)i * N + k] : 0;
    for (int jj = 0; jj < nj; ++jj) acc = addq(acc, ib[jj * sij + auto_src((u32)k, gk.g[jj], logN)], q);
    out[b * sob + (size_t)i * N + k] = acc;
}

// ModDown merged with the rescale that follows it (relinearised products at
// level l >= 1).  With FBC_i the ModDown base conversion of the P limbs (as
// k_moddown_fbc), x = [d_l + P^-1 (U_l - FBC_l)]_{q_l} the coefficient form of
// the top limb of d + ModDown(U), and c its centered residue, it writes
// Z_i = FBC_i + [P]_{q_i} [c]_{q_i} for i < l; then
// (d + ModDown(U) - NTT(c)) q_l^-1 = (d + (U - NTT(Z)) P^-1) q_l^-1 limb by limb.
// Xu: coefficient forms of U's limbs at storage index (level .. level+nP)
// in a [nE][N] layout per polynomial; Xd: coefficient form of d's limb l.
// NP > 0: compiled for exactly NP special primes (the loops over them
// unrolled without bounds tests); NP = 0: any count up to kMaxDigit
template <int NP>
__global__ __launch_bounds__(kT) void k_relin_rescale_prep(u64 *__restrict__ Z, const u64 *__restrict__ Xu,
                                                           const u64 *__restrict__ Xd, int N, int level, int nP_rt,
                                                           int pbase, int L1, const u64 *__restrict__ tab,
                                                           const ModConst *__restrict__ mods, size_t sz, size_t sxu,
                                                           size_t sxd, int no_d, const u64 *__restrict__ pbig) {
    const int nP = NP ? NP : nP_rt;
    const int k = blockIdx.x * kT + threadIdx.x, poly = blockIdx.z;
    const u64 *phat_inv = tab, *phat_inv_sh = tab + nP, *phat_mod = tab + 2 * nP;
    const u64 *pinv = tab + 2 * nP + (size_t)L1 * nP, *pinv_sh = pinv + L1;
    const u64 *pmod = pinv + 2 * L1;
    const double *invp = reinterpret_cast<const double *>(pmod + L1);
    const u64 *xu = Xu + poly * sxu + (size_t)level * N + k;
    u64 y[kMaxDigit];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kMaxDigit; ++j)
        if (j < nP) {
            y[j] = shoup(xu[(size_t)(1 + j) * N], phat_inv[j], phat_inv_sh[j], mods[pbase + j].q);
            s = s + (double)y[j] * invp[j];
        }
    const u64 e = overflow_round(y, nP, s, pbig);
    u32 y0[kMaxDigit], y1[kMaxDigit];
#pragma unroll
    for (int j = 0; j < kMaxDigit; ++j)
        if (j < nP) split30(y[j], y0[j], y1[j]);
    const u64 *epm = reinterpret_cast<const u64 *>(invp + nP);  // [L1][nP+1]: -e P 2^64 mod q_i
    auto fbc_sum = [&](int i) {
        Dot30 acc(epm[(size_t)i * (nP + 1) + e]);
#pragma unroll
        for (int j = 0; j < kMaxDigit; ++j)
            if (j < nP) acc.add(y0[j], y1[j], phat_mod[(size_t)i * nP + j]);
        return acc;
    };
    auto fbc = [&](int i, const ModConst &mi) { return fbc_sum(i).redc(mi); };
    const ModConst mt = mods[level];
    const u64 qt = mt.q;
    // folded (Xd null): limb `level` of U already holds d_l + P^-1 U_l;
    // no_d: x = P^-1 (U_l - FBC_l), the top limb of ModDown(U) alone
    u64 x;
    if (Xd || no_d) {
        x = shoup(subq(xu[0], fbc(level, mt), qt), pinv[level], pinv_sh[level], qt);
        if (Xd) x = addq(Xd[poly * sxd + k], x, qt);
    } else {
        x = subq(xu[0], shoup(fbc(level, mt), pinv[level], pinv_sh[level], qt), qt);
    }
    const bool neg = x > (qt >> 1);
    const u64 mag = neg ? qt - x : x;
    // Z_i = FBC_i + [P]_{q_i} [c]_{q_i}: the product with |c| joins the same
    // Montgomery sum, against P 2^64 (or -P 2^64) mod q_i
    const u64 *pm = epm + (size_t)L1 * (nP + 1);
    const int i0 = blockIdx.y * kFbcTargets, i1 = min(level, i0 + kFbcTargets);
    u32 m0, m1;
    split30(mag, m0, m1);
    for (int i = i0; i < i1; ++i) {
        const ModConst mi = mods[i];
        Dot30 acc = fbc_sum(i);
        acc.add(m0, m1, neg ? mi.q - pm[i] : pm[i]);
        Z[poly * sz + (size_t)i * N + k] = acc.redc(mi);
    }
}

// ModDown base conversion P -> Q_level of the P limbs in coefficient form,
// to the CENTERED residue of u mod P: y_j = [u_j * Phat_j^-1]_{p_j},
// X = sum_j y_j Phat_j in [0, nP P), e = round(X / P) (overflow_round: FP64
// estimate, decided in integers near a half-integer), and
// V_i = (sum_j y_j [Phat_j]_{q_i} - e [P]_{q_i}) mod q_i.
// tab: phat_inv[nP], phat_inv_sh[nP], phat_mod[(L+1)][nP], Pinv[L+1],
//      Pinv_sh[L+1], P_mod_q[L+1], inv_p[nP] (double bits)
template <int NP>
__global__ __launch_bounds__(kT) void k_moddown_fbc(u64 *__restrict__ V, const u64 *__restrict__ Upc, int N, int level,
                                                    int nP_rt, int pbase, int L1, const u64 *__restrict__ tab,
                                                    const ModConst *__restrict__ mods, size_t sv, size_t su,
                                                    const u64 *__restrict__ pbig) {
    const int nP = NP ? NP : nP_rt;
    const int k = blockIdx.x * kT + threadIdx.x, poly = blockIdx.z;
    const u64 *phat_inv = tab, *phat_inv_sh = tab + nP, *phat_mod = tab + 2 * nP;
    const u64 *pmod = tab + 2 * nP + (size_t)L1 * nP + 2 * L1;
    const double *invp = reinterpret_cast<const double *>(pmod + L1);
    u64 y[kMaxDigit];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kMaxDigit; ++j)
        if (j < nP) {
            y[j] = shoup(Upc[poly * su + (size_t)j * N + k], phat_inv[j], phat_inv_sh[j], mods[pbase + j].q);
            s = s + (double)y[j] * invp[j];
        }
    const u64 e = overflow_round(y, nP, s, pbig);
    u32 y0[kMaxDigit], y1[kMaxDigit];
#pragma unroll
    for (int j = 0; j < kMaxDigit; ++j)
        if (j < nP) split30(y[j], y0[j], y1[j]);
    const u64 *epm = reinterpret_cast<const u64 *>(invp + nP);  // [L1][nP+1]: -e P 2^64 mod q_i
    const int i0 = blockIdx.y * kFbcTargets, i1 = min(level + 1, i0 + kFbcTargets);
    for (int i = i0; i < i1; ++i) {
        Dot30 acc(epm[(size_t)i * (nP + 1) + e]);
#pragma unroll
        for (int j = 0; j < kMaxDigit; ++j)
            if (j < nP) acc.add(y0[j], y1[j], phat_mod[(size_t)i * nP + j]);
        V[poly * sv + (size_t)i * N + k] = acc.redc(mods[i]);
    }
}

// U[p] limb `level` <- d[p] limb level + P^-1 U[p] limb level (the top-limb
// fold that the relinearisation key inner product applies in its epilogue)
__global__ __launch_bounds__(kT) void k_fold_top(u64 *U, const u64 *d, int N, int level, u64 pinv, u64 pinv_sh,
                                                 const ModConst *mods, size_t su, size_t sd) {
    const int k = blockIdx.x * kT + threadIdx.x, p = blockIdx.z;
    const u64 q = mods[level].q;
    u64 *u = U + p * su + (size_t)level * N + k;
    *u = addq(d[p * sd + (size_t)level * N + k], shoup(*u, pinv, pinv_sh, q), q);
}

__global__ __launch_bounds__(kT) void k_moddown_finish(u64 *out, const u64 *U, const u64 *V, int N, const u64 *pinv,
                                                       const u64 *pinv_sh, const ModConst *mods, size_t so,
                                                       size_t su, size_t sv, int accumulate) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z;
    const u64 q = mods[i].q;
    const size_t w = (size_t)i * N + k;
    u64 r = shoup(subq(U[p * su + w], V[p * sv + w], q), pinv[i], pinv_sh[i], q);
    if (accumulate) r = addq(r, out[p * so + w], q);
    out[p * so + w] = r;
}

// Y[p][i] = centered(x_p) mod q_i, i < level; x_p canonical mod q_level
__global__ __launch_bounds__(kT) void k_rescale_prep(u64 *Y, const u64 *xtop, int N, int level, size_t sy,
                                                     size_t sx, const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z;
    const u64 ql = mods[level].q;
    const ModConst mi = mods[i];
    const u64 x = xtop[p * sx + k];
    u64 v;
    if (x > (ql >> 1)) {
        const u64 neg = reduce64(ql - x, mi);
        v = neg ? mi.q - neg : 0;
    } else {
        v = reduce64(x, mi);
    }
    Y[p * sy + (size_t)i * N + k] = v;
}

__global__ __launch_bounds__(kT) void k_rescale_finish(u64 *out, const u64 *in, const u64 *Y, int N, const u64 *qinv,
                                                       const u64 *qinv_sh, const ModConst *mods, size_t so,
                                                       size_t si, size_t sy) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z;
    const u64 q = mods[i].q;
    const size_t w = (size_t)i * N + k;
    out[p * so + w] = shoup(subq(in[p * si + w], Y[p * sy + w], q), qinv[i], qinv_sh[i], q);
}

constexpr int kMacQ = 8;  // queries per MAC launch (baby pointer table in the kernel arguments)
struct BabyPtrs {
    const u64 *p[kMacQ][32];
    const unsigned char *diag[kMacQ];  // diagonal group of each query
};

// one diagonal word: a 64-bit limb, or a packed limb's low word and high byte
template <bool PK>
__device__ __forceinline__ u64 diag_word(const unsigned char *limb, size_t off, int k, int N) {
    if (PK)
        return (u64)reinterpret_cast<const u32 *>(limb + off)[k] | ((u64)(limb + off + 4 * (size_t)N)[k] << 32);
    return reinterpret_cast<const u64 *>(limb + off)[k];
}

// b = e - a s + [limb in digit] (P mod q) s'   (key generation, eval domain;
// limbs are global modulus indices; s_mont Montgomery-scaled)
__global__ __launch_bounds__(kT) void k_key_combine(u64 *b, const u64 *a, const u64 *e, const u64 *s_mont,
                                                    const u64 *sp, LimbConsts pm, int dlo, int dhi, int N,
                                                    const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const ModConst m = mods[i];
    const size_t w = (size_t)i * N + k;
    const u64 x = a[w];
    u64 r = subq(e[w], redc(x * s_mont[w], mulhi64(x, s_mont[w]), m), m.q);
    if (sp && i >= dlo && i < dhi) r = addq(r, shoup(sp[w], pm.v[i], pm.sh[i], m.q), m.q);
    b[w] = r;
}

// c0 = v b + e0 + m, c1 = v a + e1 (encryption, eval domain)
__global__ __launch_bounds__(kT) void k_encrypt_combine(u64 *c0, u64 *c1, const u64 *v, const u64 *e0, const u64 *e1,
                                                        const u64 *msg, const u64 *pkb, const u64 *pka, int N,
                                                        const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const ModConst m = mods[i];
    const size_t w = (size_t)i * N + k;
    const u64 vv = v[w];
    c0[w] = addq(addq(mulmod(vv, pkb[w], m), e0[w], m.q), msg[w], m.q);
    c1[w] = addq(mulmod(vv, pka[w], m), e1[w], m.q);
}

// m = c0 + c1 s (decryption, eval domain; s_mont Montgomery-scaled)
__global__ __launch_bounds__(kT) void k_decrypt_combine(u64 *out, const u64 *c0, const u64 *c1, const u64 *s_mont,
                                                        int N, const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const ModConst m = mods[i];
    const size_t w = (size_t)i * N + k;
    const u64 x = c1[w], s = s_mont[w];
    out[w] = addq(c0[w], redc(x * s, mulhi64(x, s), m), m.q);
}


// Fused multiply-accumulate of the BSGS inner sums (Eq. bsgs2):
//   P_j[c][m][k] = sum_i baby_i[c][m][k] * diag_{j n1 + i}[m][k]
// A wave covers 32 coefficients of one limb for both polynomials (lanes
// 0..31: c0, lanes 32..63: c1), so each diagonal word is fetched once per
// wave and shared by the two half-waves.  Positions past ell or nj are
// staged as zero words and contribute nothing (a launch whose tile lies
// inside the matrix is compiled without those guards).  The diagonals are
// Montgomery-scaled by 2^64, so each sum, held exactly, takes one Montgomery
// reduction at the end; at most 32 terms per launch.
//
// 64-bit limbs: 128-bit lazy sums of full products (each below 2^122).
// Packed limbs (q < 2^40, diagonal word w = wl + wh 2^32 with wh < 2^8; baby
// word b below 2^45, canonical words are below q): with b = b0 + b1 2^27
// (b0 < 2^27, b0s = b0 2^5), the product splits as
//   b w = b0 wl + 2^27 (b1 wl + b0s wh) + 2^59 b1 wh,
// three sums that cannot overflow their words over 32 terms (below 2^64,
// 2^56 and 2^32): three 32 x 32 -> 64-bit and one 24-bit multiply-add per
// term in place of a full 64 x 64 product and its carries.
// P_j = (hi:lo) 2^-64 mod q (+ P_j) for the tile's giant steps.  The sums
// are written with non-temporal stores: they are not read again by this
// launch, and streaming them past the caches keeps the write-backs from
// interleaving with the diagonal stream (measured: 7% less MAC time).
template <int NJ>
__device__ __forceinline__ void mac3_store(u64 *P, const u64 *lo, const u64 *hi, int j0, int nj, int p, int lv, int m,
                                           int N, int k, const ModConst &mc, int accumulate) {
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        if (jj < nj) {
            const size_t o = (((size_t)(j0 + jj) * 2 + p) * (lv + 1) + m) * N + k;
            u64 r = redc_any(lo[jj], hi[jj], mc);
            if (accumulate) r = addq(r, P[o], mc.q);
            __builtin_nontemporal_store(r, &P[o]);
        }
    }
}


// stage stride of the MAC's LDS tile (NJ diagonal slices and two baby
// limbs, in whole 1 KiB chunks)
template <int NJ, bool PK>
constexpr int mac3_stage_bytes() {
    return ((NJ * (PK ? 640 : 1024) + 2048 + 1023) / 1024) * 1024;
}

// The words of a block's tile go through LDS: for each baby step the
// block's slice of its NJ diagonals (128 coefficients each: 512 low-word
// bytes and 128 high bytes of a packed limb, or 1 KiB) and of the baby
// step's c0 and c1 limbs (1 KiB each) is copied from HBM straight into one
// of two LDS stages, one baby step ahead, by wave-wide 16-byte loads that
// write LDS without passing through registers (global_load_lds_dwordx4: lane
// l of a load lands at byte 16 l of its 1 KiB chunk), and read from there by
// the lanes (the c0 and the c1 half-wave read the same diagonal words).
// Such loads are counted by vmcnt, so the barrier's wait for vmcnt(0)
// publishes a stage to the block.  Staging through registers instead costs
// about 20 registers per lane and an LDS write pass, and per-lane 4-byte and
// 1-byte loads of the same bytes stream at about two thirds of the rate of
// 16-byte loads.
template <int NJ, bool FULL, bool PK>
__device__ __forceinline__ void mac3_body(u64 *P, size_t pq, const BabyPtrs &bp, int nq, int q, int tile, int m, int nb,
                                          int i0, int n1, int j0, int nj, int ell, size_t dstride, unsigned loff,
                                          int bl, int lv, int N, const ModConst &mc, int accumulate,
                                          unsigned char *lds) {
    constexpr int SLOT = PK ? 640 : 1024;  // bytes of one diagonal's slice of the tile
    constexpr int U4 = SLOT / 16, TOT = NJ * U4 + 128;  // 16-byte pieces of a stage
    constexpr int NCH = (TOT + 63) / 64, STG = NCH * 1024;  // 1 KiB chunks (one wave-wide load each), stage stride
    static_assert(STG == mac3_stage_bytes<NJ, PK>(), "stage stride");
    constexpr int BABY = NJ * SLOT;  // the stage's baby slice (c0 then c1, 1 KiB each) follows the diagonals'
    const int t = threadIdx.x, lane = t & 63, p = lane >> 5, wv = t >> 6;
    const int kk = wv * 32 + (lane & 31), k0 = tile * (kT / 2), k = k0 + kk;
    const unsigned char *dg = bp.diag[q] + loff;
    // diagonal (j0 + jj) n1 + i0 + ii at base + ii dstride + jj jstride
    const unsigned char *base = dg + ((size_t)j0 * n1 + i0) * dstride;
    const size_t jstride = (size_t)n1 * dstride;
    P += q * pq;
    // baby step ii's pieces into stage b: chunk c is loaded by wave c mod 4,
    // its lane l carrying piece 64 c + l (diagonal pieces, then the baby
    // step's two limbs, then zero padding up to a whole chunk)
    auto dma = [&](int ii, int b) {
        unsigned char *dst = lds + b * STG;
        const unsigned char *bl0 = reinterpret_cast<const unsigned char *>(bp.p[q][ii]);
#pragma unroll
        for (int c = wv; c < NCH; c += kT / 64) {
            const int i = c * 64 + lane;
            const void *src = &g_zero16;
            if (i >= NJ * U4 && i < TOT) {
                const int w = i - NJ * U4, pb = w >> 6;
                src = bl0 + (((size_t)pb * (bl + 1) + m) * N + k0) * 8 + 16 * (w & 63);
            } else if (i < TOT) {
                const int jj = i / U4, w = i - jj * U4;
                if (FULL || (jj < nj && (j0 + jj) * n1 + i0 + ii < ell)) {
                    const unsigned char *row = base + (size_t)ii * dstride + jj * jstride;
                    src = !PK ? row + 8 * (size_t)k0 + 16 * w
                        : w < 32 ? row + 4 * (size_t)k0 + 16 * w
                                 : row + 4 * (size_t)N + k0 + 16 * (w - 32);
                }
            }
            if (nq == 1)
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(dst + c * 1024), 16,
                                                 0, kCachePolicyNT);
            else  // the blocks of the launch's queries share each tile through the L2
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(dst + c * 1024), 16,
                                                 0, 0);
        }
    };
    auto baby = [&](int ii) {
        return reinterpret_cast<const u64 *>(lds + (ii & 1) * STG + BABY + p * 1024)[kk];
    };
    // stage ii complete for the whole block (this wave's loads: vmcnt(0);
    // the other waves': the barrier), and every wave done with stage ii - 1
    auto publish = [&]() {
        __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0)
        __syncthreads();
    };
    dma(0, 0);
    if constexpr (PK) {
        // A = sum b0 wl, Bm = sum (b1 wl + b0s wh), D = sum b1 wh
        u64 A[NJ], Bm[NJ];
        u32 D[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) A[jj] = Bm[jj] = 0, D[jj] = 0;
        for (int ii = 0; ii < nb; ++ii) {
            publish();
            if (ii + 1 < nb) dma(ii + 1, (ii + 1) & 1);
            const u64 b = baby(ii);
            const unsigned char *st = lds + (ii & 1) * STG;
            const u32 b0 = (u32)b & 0x7ffffffu, b1 = (u32)(b >> 27) & 0xffffffu, b0s = b0 << 5;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const u32 wl = reinterpret_cast<const u32 *>(st + jj * SLOT)[kk];
                const u32 wh = st[jj * SLOT + 512 + kk];
                A[jj] += (u64)b0 * wl;
                Bm[jj] += (u64)b1 * wl;
                Bm[jj] += (u64)b0s * wh;
                D[jj] += b1 * wh;
            }
        }
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const unsigned __int128 s =
                (unsigned __int128)A[jj] + ((unsigned __int128)Bm[jj] << 27) + ((unsigned __int128)D[jj] << 59);
            A[jj] = (u64)s;
            Bm[jj] = (u64)(s >> 64);
        }
        mac3_store<NJ>(P, A, Bm, j0, nj, p, lv, m, N, k, mc, accumulate);
    } else {
        unsigned __int128 acc[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) acc[jj] = 0;
        for (int ii = 0; ii < nb; ++ii) {
            publish();
            if (ii + 1 < nb) dma(ii + 1, (ii + 1) & 1);
            const u64 b = baby(ii);
            const unsigned char *st = lds + (ii & 1) * STG;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj)
                acc[jj] += (unsigned __int128)b * reinterpret_cast<const u64 *>(st + jj * SLOT)[kk];
        }
        u64 lo[NJ], hi[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) lo[jj] = (u64)acc[jj], hi[jj] = (u64)(acc[jj] >> 64);
        mac3_store<NJ>(P, lo, hi, j0, nj, p, lv, m, N, k, mc, accumulate);
    }
}

template <int NJ, bool FULL, bool PK>
__global__ __launch_bounds__(kT) void k_bsgs_mac3(u64 *P, size_t pq, BabyPtrs bp, int nq, int nb, int i0, int n1, int j0,
                                                  int nj, int ell, size_t dstride, DbLayout lay, int bl, int lv, int N,
                                                  const ModConst *mods, int accumulate, int lq, int pofs,
                                                  unsigned sel) {
    __shared__ __align__(16) unsigned char lds[2 * mac3_stage_bytes<NJ, PK>()];
    int q, tile;
    item_tile(blockIdx.x, nq, N / (kT / 2), q, tile);
    // limb m: the (blockIdx.y + 1)-th set bit of sel (wave-uniform scalar work)
    for (unsigned y = blockIdx.y; y; --y) sel &= sel - 1;
    const int m = __builtin_ctz(sel);
    const ModConst mc = mods[m <= lq ? m : m + pofs];
    mac3_body<NJ, FULL, PK>(P, pq, bp, nq, q, tile, m, nb, i0, n1, j0, nj, ell, dstride, lay.off[m], bl, lv, N, mc,
                            accumulate, lds);
}

// The hoisted product's baby steps formed inside the MAC (Eq. bsgs2 with
// the key inner products of the hoisted rotations, §3.4.2): the words of
// baby step i >= 1 are never written to memory.  A block's 128 outputs
// k0 .. k0+127 of limb m take their sources, under every rotation, from
// one aligned 128-word block S0 .. S0+127 (the automorphism maps aligned
// 128-word blocks onto aligned 128-word blocks), so a stage carries, after
// the NJ diagonal slices, that block of each of the ND ModUp digits and of
// c0, and the 2 ND key slices of the outputs (digit t, part b then a).
// Lane (k, c) forms
//   b = [sum_t D_t[m][s] ksk_{i,t,c}[m][k] + (c = 0, m <= l) P c0[m][s]] 2^-64 mod q_m
// with s = auto_src(k, g_i): the word the separate key inner product writes
// for the baby step (same exact sum, same reduction), then accumulates it
// against the diagonals as the MAC does.  Baby step 0 (P times the query)
// is formed the same way from the query's words.  One launch covers n1 <= 32 baby steps, every giant
// step of the tile inside the matrix (NJ = 16), packed or 64-bit limbs.
struct KsMacSrc {
    const unsigned char *diag[kMacQ];  // diagonal group of each query
    const unsigned char *ksk[32];      // key of baby step i (i >= 1)
    u64 g[32];                         // Galois element of baby step i
};
// A stage is made of whole 1 KiB chunks, each filled by one wave-wide
// global-to-LDS load (lane l: bytes 16 l .. 16 l + 15) and each holding one
// kind of word, so the wave that loads a chunk takes one scalar branch:
//   diagonals: packed: 8 chunks of low words (slices 2c, 2c+1), 2 chunks of
//     high bytes (8 slices each); 64-bit: one chunk per slice;
//   then, for baby step 0: the query's c0 and c1 slices; for baby step i >= 1: the
//     ND digit blocks, the c0 block, and the key slices (digit t's parts b
//     and a at slices 2t, 2t+1): packed: ND chunks of low words and one of
//     high bytes; 64-bit: one chunk per slice.
template <int NJ, bool PK, int ND>
struct KsMacShape {
    static constexpr int CDL = PK ? NJ / 2 : NJ;              // chunks of diagonal low words / 64-bit slices
    static constexpr int CD = PK ? CDL + NJ / 8 : NJ;         // diagonal chunks
    static constexpr int CX = PK ? 2 * ND + 2 : 3 * ND + 1;   // chunks of a baby step i >= 1
    static constexpr int NCH = CD + CX;
    static constexpr int STG = NCH * 1024;
    static_assert(NJ % 8 == 0 && CX >= 2, "chunk layout");
};
template <int NJ, bool PK, int ND>
constexpr int ksmac_stage_bytes() {
    return KsMacShape<NJ, PK, ND>::STG;
}
template <int NJ, bool PK, int ND>
__device__ __forceinline__ void ksmac_body(u64 *P, size_t pq, const KsMacSrc &ks, int nq, int q, int tile, int m, int nb,
                                           int n1, size_t dstride, unsigned loff, const u64 *D, size_t sd,
                                           const u64 *C, size_t sc, unsigned koff, size_t kblock, int nE, int lq,
                                           int logN, int N, u64 pm, const ModConst &mc, unsigned char *lds) {
    using S = KsMacShape<NJ, PK, ND>;
    constexpr int STG = S::STG, RX = S::CD * 1024;
    const int t = threadIdx.x, lane = t & 63, p = lane >> 5;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int kk = wv * 32 + (lane & 31), k0 = tile * (kT / 2), k = k0 + kk;
    const unsigned char *base = ks.diag[q] + loff;
    const size_t jstride = (size_t)n1 * dstride;
    P += q * pq;
    const unsigned char *Db = reinterpret_cast<const unsigned char *>(D + q * sd);
    const unsigned char *Cb = reinterpret_cast<const unsigned char *>(C + q * sc);
    auto dma = [&](int ii, int b) {
        unsigned char *dst = lds + b * STG;
        const u32 S0 = ii ? auto_src((u32)k0, ks.g[ii], logN) & ~127u : 0u;
        const unsigned char *kl0 = ks.ksk[ii] + koff;
        const unsigned char *drow = base + (size_t)ii * dstride;
#pragma unroll
        for (int c = wv; c < S::NCH; c += kT / 64) {
            const void *src = nullptr;
            if (c < S::CD) {
                if (PK) {
                    if (c < S::CDL)
                        src = drow + (2 * c + (lane >> 5)) * jstride + 4 * (size_t)k0 + 16 * (lane & 31);
                    else
                        src = drow + (8 * (c - S::CDL) + (lane >> 3)) * jstride + 4 * (size_t)N + k0 + 16 * (lane & 7);
                } else {
                    src = drow + c * jstride + 8 * (size_t)k0 + 16 * lane;
                }
            } else {
                const int x = c - S::CD;
                if (ii == 0) {
                    // the query's c0 and c1 slices (limbs up to l)
                    if (x < 2 && m <= lq) src = Cb + (((size_t)x * (lq + 1) + m) * N + k0) * 8 + 16 * lane;
                } else if (x < ND) {
                    src = Db + (((size_t)x * nE + m) * N + S0) * 8 + 16 * lane;
                } else if (x == ND) {
                    if (m <= lq) src = Cb + ((size_t)m * N + S0) * 8 + 16 * lane;
                } else if (PK) {
                    const int kx = x - ND - 1;
                    if (kx < ND)
                        src = kl0 + (size_t)(2 * kx + (lane >> 5)) * kblock + 4 * (size_t)k0 + 16 * (lane & 31);
                    else if (lane < 2 * ND * 8)
                        src = kl0 + (size_t)(lane >> 3) * kblock + 4 * (size_t)N + k0 + 16 * (lane & 7);
                } else {
                    src = kl0 + (size_t)(x - ND - 1) * kblock + 8 * (size_t)k0 + 16 * lane;
                }
            }
            if (!src) continue;
            auto *d = (__attribute__((address_space(3))) void *)(dst + c * 1024);
            // the diagonals and keys are read once: non-temporal for one
            // query; the digit and c0 blocks come back under every rotation
            if (nq == 1 && (c < S::CD || c > S::CD + ND))
                __builtin_amdgcn_global_load_lds(src, d, 16, 0, kCachePolicyNT);
            else
                __builtin_amdgcn_global_load_lds(src, d, 16, 0, 0);
        }
    };
    // this lane's word of baby step ii (stage ii & 1); a c0 block left
    // unloaded (limbs past l) only meets the weight 0
    auto baby = [&](int ii) -> u64 {
        const unsigned char *x = lds + (ii & 1) * STG + RX;
        if (ii == 0) {
            // baby step 0 = P times the query: P 2^64 (the weight pm) times
            // the word, one reduction; 0 on the special primes
            if (pm == 0) return 0;
            u32 y0, y1;
            split30(reinterpret_cast<const u64 *>(x + p * 1024)[kk], y0, y1);
            Dot30 s0;
            s0.add(y0, y1, pm);
            return s0.redc(mc);
        }
        const u32 S0 = auto_src((u32)k0, ks.g[ii], logN) & ~127u;
        const u32 r = auto_src((u32)k, ks.g[ii], logN) - S0;
        const unsigned char *kx = x + (ND + 1) * 1024;
        Dot30 s;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            u32 y0, y1;
            split30(reinterpret_cast<const u64 *>(x + d * 1024)[r], y0, y1);
            const int li = 2 * d + p;
            const u64 w = PK ? ((u64)reinterpret_cast<const u32 *>(kx + li * 512)[kk] |
                                ((u64)kx[ND * 1024 + li * 128 + kk] << 32))
                             : reinterpret_cast<const u64 *>(kx + li * 1024)[kk];
            s.add(y0, y1, w);
        }
        u32 c00, c01;
        split30(reinterpret_cast<const u64 *>(x + ND * 1024)[r], c00, c01);
        s.add(c00, c01, p == 0 ? pm : 0);
        return s.redc(mc);
    };
    auto publish = [&]() {
        __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0)
        __syncthreads();
    };
    dma(0, 0);
    if constexpr (PK) {
        u64 A[NJ], Bm[NJ];
        u32 Dh[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) A[jj] = Bm[jj] = 0, Dh[jj] = 0;
        for (int ii = 0; ii < nb; ++ii) {
            publish();
            if (ii + 1 < nb) dma(ii + 1, (ii + 1) & 1);
            const u64 b = baby(ii);
            const unsigned char *st = lds + (ii & 1) * STG;
            const u32 b0 = (u32)b & 0x7ffffffu, b1 = (u32)(b >> 27) & 0xffffffu, b0s = b0 << 5;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const u32 wl = reinterpret_cast<const u32 *>(st + jj * 512)[kk];
                const u32 wh = st[S::CDL * 1024 + jj * 128 + kk];
                A[jj] += (u64)b0 * wl;
                Bm[jj] += (u64)b1 * wl;
                Bm[jj] += (u64)b0s * wh;
                Dh[jj] += b1 * wh;
            }
        }
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const unsigned __int128 x =
                (unsigned __int128)A[jj] + ((unsigned __int128)Bm[jj] << 27) + ((unsigned __int128)Dh[jj] << 59);
            A[jj] = (u64)x;
            Bm[jj] = (u64)(x >> 64);
        }
        mac3_store<NJ>(P, A, Bm, 0, NJ, p, nE - 1, m, N, k, mc, 0);
    } else {
        unsigned __int128 acc[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) acc[jj] = 0;
        for (int ii = 0; ii < nb; ++ii) {
            publish();
            if (ii + 1 < nb) dma(ii + 1, (ii + 1) & 1);
            const u64 b = baby(ii);
            const unsigned char *st = lds + (ii & 1) * STG;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj)
                acc[jj] += (unsigned __int128)b * reinterpret_cast<const u64 *>(st + jj * 1024)[kk];
        }
        u64 lo[NJ], hi[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) lo[jj] = (u64)acc[jj], hi[jj] = (u64)(acc[jj] >> 64);
        mac3_store<NJ>(P, lo, hi, 0, NJ, p, nE - 1, m, N, k, mc, 0);
    }
}

template <int NJ, bool PK, int ND>
__global__ __launch_bounds__(kT) void k_bsgs_ksmac(u64 *P, size_t pq, KsMacSrc ks, int nq, int nb, int n1,
                                                   size_t dstride, DbLayout lay, KeyLayout kl, const u64 *D,
                                                   size_t sd, const u64 *C, size_t sc, int nE, int lq, int pofs,
                                                   int logN, int N, const ModConst *mods, const u64 *pmont,
                                                   unsigned sel) {
    __shared__ __align__(16) unsigned char lds[2 * ksmac_stage_bytes<NJ, PK, ND>()];
    int q, tile;
    item_tile(blockIdx.x, nq, N / (kT / 2), q, tile);
    for (unsigned y = blockIdx.y; y; --y) sel &= sel - 1;
    const int m = __builtin_ctz(sel);
    const int gm = m <= lq ? m : m + pofs;
    const ModConst mc = mods[gm];
    const u64 pm = m <= lq ? pmont[m] : 0;
    ksmac_body<NJ, PK, ND>(P, pq, ks, nq, q, tile, m, nb, n1, dstride, lay.off[m], D, sd, C, sc, kl.off[gm], kl.block,
                           nE, lq, logN, N, pm, mc, lds);
}

// 64-bit limbs <-> the packed diagonal layout (grid: N / kT, nl, nd)
__global__ __launch_bounds__(kT) void k_db_pack(unsigned char *dst, size_t dstride, DbLayout lay, const u64 *src,
                                                int nl, int N) {
    const int k = blockIdx.x * kT + threadIdx.x, m = blockIdx.y, d = blockIdx.z;
    const u64 x = src[((size_t)d * nl + m) * N + k];
    unsigned char *limb = dst + d * dstride + lay.off[m];
    if (lay.packed[m]) {
        reinterpret_cast<u32 *>(limb)[k] = (u32)x;
        limb[4 * (size_t)N + k] = (unsigned char)(x >> 32);
    } else {
        reinterpret_cast<u64 *>(limb)[k] = x;
    }
}
__global__ __launch_bounds__(kT) void k_db_unpack(u64 *dst, const unsigned char *src, size_t sstride, DbLayout lay,
                                                  int nl, int N) {
    const int k = blockIdx.x * kT + threadIdx.x, m = blockIdx.y, d = blockIdx.z;
    const unsigned char *limb = src + d * sstride + lay.off[m];
    dst[((size_t)d * nl + m) * N + k] = lay.packed[m] ? diag_word<true>(limb, 0, k, N) : diag_word<false>(limb, 0, k, N);
}

// key blocks between 64-bit limbs [nb][nm][N] and the KeyLayout bytes
// (grid: N / kT, nm, nb)
__global__ __launch_bounds__(kT) void k_key_pack(unsigned char *dst, KeyLayout kl, const u64 *src, int nm, int N) {
    const int k = blockIdx.x * kT + threadIdx.x, m = blockIdx.y, b = blockIdx.z;
    const u64 x = src[((size_t)b * nm + m) * N + k];
    unsigned char *limb = dst + b * kl.block + kl.off[m];
    if (kl.packed[m]) {
        reinterpret_cast<u32 *>(limb)[k] = (u32)x;
        limb[4 * (size_t)N + k] = (unsigned char)(x >> 32);
    } else {
        reinterpret_cast<u64 *>(limb)[k] = x;
    }
}
__global__ __launch_bounds__(kT) void k_key_unpack(u64 *dst, KeyLayout kl, const unsigned char *src, int nm, int N) {
    const int k = blockIdx.x * kT + threadIdx.x, m = blockIdx.y, b = blockIdx.z;
    const unsigned char *limb = src + b * kl.block + kl.off[m];
    dst[((size_t)b * nm + m) * N + k] = kl.packed[m] ? key_word<true>(limb, k, N) : key_word<false>(limb, k, N);
}

// out_b[i][p] = (U_b[i][p] - V_b[i][p]) P^-1 + in_b[i][auto_src(p, g)]: the
// ModDown finish of one rotation of several ciphertexts fused with the
// automorphism of c0 (c1 part: no add).  U_b, V_b are consecutive items.
constexpr int kRotItems = 16;
struct RotItems {
    u64 *out[kRotItems];
    const u64 *in[kRotItems];
};
__global__ __launch_bounds__(kT) void k_moddown_rot(RotItems it, const u64 *__restrict__ U, const u64 *__restrict__ V, u64 g, int N, int logN,
                                                    int lp1, const u64 *__restrict__ pinv, const u64 *__restrict__ pinv_sh, const ModConst *__restrict__ mods,
                                                    size_t su) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, p = blockIdx.z & 1, b = blockIdx.z >> 1;
    const u64 q = mods[i].q;
    const size_t w = (size_t)i * N + k;
    const size_t lw = (size_t)lp1 * N;
    u64 r = shoup(subq(U[(2 * b + p) * su + w], V[(2 * b + p) * lw + w], q), pinv[i], pinv_sh[i], q);
    if (p == 0) r = addq(r, it.in[b][(size_t)i * N + auto_src((u32)k, g, logN)], q);
    it.out[b][p * lw + w] = r;
}

// ---------------------------------------------------------------------------
// batched element-wise kernels of the Chebyshev waves: per-item pointers and
// constants travel in the kernel arguments (up to kBatch items per launch)
// ---------------------------------------------------------------------------
constexpr int kBatch = 16, kTerms = 8;
static_assert(kRotItems == kBatch, "one item limit for the pointer-table launches");

__device__ __forceinline__ u64 smod_dev(long long v, const ModConst &m) {
    if (v >= 0) return reduce64((u64)v, m);
    const u64 a = reduce64((u64)(-(v + 1)), m);  // -(v+1) >= 0 avoids overflow
    const u64 b = a + 1 == m.q ? 0 : a + 1;
    return b ? m.q - b : 0;
}

struct ScalarBatch {
    const u64 *src[kBatch][kTerms];
    long long k[kBatch][kTerms];
    int src_lp1[kBatch][kTerms];  // (level + 1) of each source: its polynomial stride in limbs
    int nterms[kBatch];
    int accumulate;  // add to the current output instead of overwriting it
};

// out_b (+)= sum_t k_{b,t} * src_{b,t} over the first nl limbs of both
// polynomials; out items are contiguous [B][2][nl][N]
__global__ __launch_bounds__(kT) void k_scalar_batch(u64 *out, ScalarBatch sb, int nl, int N, const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y % nl, p = blockIdx.y / nl, b = blockIdx.z;
    const ModConst m = mods[i];
    u64 *o = out + (((size_t)b * 2 + p) * nl + i) * N + k;
    u64 acc = sb.accumulate ? *o : 0;
    for (int t = 0; t < sb.nterms[b]; ++t) {
        const u64 x = sb.src[b][t][((size_t)p * sb.src_lp1[b][t] + i) * N + k];
        acc = addq(acc, mulmod(x, smod_dev(sb.k[b][t], m), m), m.q);
    }
    *o = acc;
}

// Scalar combinations sharing their sources (a wave of Chebyshev leaves,
// scalars and level adjustments): for query q (blockIdx.z) and output b,
//   out[b][q] = sum_s K[b][s] src[q][s]   on the first nl limbs of both polynomials,
// K small signed integers, reduced per limb and Montgomery-scaled into LDS
// by the block (as 30-bit halves).  A thread reads its word of every source
// once, then forms each output as an exact sum of at most kMatS products
// (Dot30), reduced once; zero entries are skipped by a per-output bit mask
// (uniform).
constexpr int kMatS = 16, kMatB = 16, kMatQ = 8;
struct ScalarMat {
    const u64 *src[kMatQ][kMatS];
    int lp1[kMatS];  // (level + 1) of each source: its polynomial stride in limbs
    long long k[kMatB][kMatS];
    unsigned nz[kMatB];  // bit s: K[b][s] != 0
    int ns, nb;
};
__global__ __launch_bounds__(kT) void k_scalar_mat(u64 *out, size_t ob, size_t oq, ScalarMat sm, int nl, int N,
                                                   const ModConst *mods) {
    __shared__ u64 kc[kMatB * kMatS];
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y % nl, p = blockIdx.y / nl, q = blockIdx.z;
    const ModConst m = mods[i];
    for (int t = threadIdx.x; t < kMatB * kMatS; t += kT) {
        const int b = t / kMatS, s = t % kMatS;
        const u64 w = (b < sm.nb && s < sm.ns) ? shoup(smod_dev(sm.k[b][s], m), m.r64, m.r64_sh, m.q) : 0;
        kc[t] = (w >> 30) << 32 | (w & 0x3fffffffu);  // its 30-bit halves
    }
    u32 x0[kMatS], x1[kMatS];
#pragma unroll
    for (int s = 0; s < kMatS; ++s)
        split30(s < sm.ns ? sm.src[q][s][((size_t)p * sm.lp1[s] + i) * N + k] : 0, x0[s], x1[s]);
    __syncthreads();
    u64 *o = out + q * oq + ((size_t)p * nl + i) * N + k;
    for (int b = 0; b < sm.nb; ++b) {
        const unsigned nz = sm.nz[b];
        Dot30 acc;
#pragma unroll
        for (int s = 0; s < kMatS; ++s)
            if (nz >> s & 1u) {
                const u64 w = kc[b * kMatS + s];
                acc.add(x0[s], x1[s], (u32)w, (u32)(w >> 32));
            }
        o[b * ob] = acc.redc(m);
    }
}

// c0 of item b (items [B][2][nl][N]) gets the constant v_b on every word
struct ConstBatch {
    long long v[kBatch];
};
__global__ __launch_bounds__(kT) void k_add_const_batch(u64 *data, ConstBatch cb, int nl, int N, size_t item,
                                                        const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, b = blockIdx.z;
    if (cb.v[b] == 0) return;
    const ModConst m = mods[i];
    u64 &x = data[b * item + (size_t)i * N + k];
    x = addq(x, smod_dev(cb.v[b], m), m.q);
}

struct PairBatch {
    const u64 *a[kBatch];
    const u64 *b[kBatch];
    u64 *out[kBatch];
    long long cst[kBatch];  // added to c0 after the operation (0: none)
    int op[kBatch];         // 0 add, 1 sub, 2 twice a minus b
};
// out_b = a_b + b_b, a_b - b_b or 2 a_b - b_b (+ cst_b on c0), ciphertexts of nl
// limbs per polynomial
__global__ __launch_bounds__(kT) void k_pair_batch(PairBatch pb, int nl, int N, const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y % nl, p = blockIdx.y / nl, b = blockIdx.z;
    const ModConst m = mods[i];
    const size_t w = ((size_t)p * nl + i) * N + k;
    const u64 x = pb.a[b][w], y = pb.b[b][w];
    const int op = pb.op[b];
    u64 r = op == 0 ? addq(x, y, m.q) : subq(op == 2 ? addq(x, x, m.q) : x, y, m.q);
    if (p == 0 && pb.cst[b]) r = addq(r, smod_dev(pb.cst[b], m), m.q);
    pb.out[b][w] = r;
}

struct TensorBatch {
    const u64 *a[kBatch];
    const u64 *b[kBatch];
};
// item b: d0, d1 into t01 + b * 2 lw, d2 into t2 + b * lw
__global__ __launch_bounds__(kT) void k_tensor_batch(u64 *t01, u64 *t2, TensorBatch tb, int nl, int N,
                                                     const ModConst *mods) {
    const int k = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, b = blockIdx.z;
    const ModConst m = mods[i];
    const size_t lw = (size_t)nl * N, w = (size_t)i * N + k;
    const u64 x0 = tb.a[b][w], x1 = tb.a[b][lw + w], y0 = tb.b[b][w], y1 = tb.b[b][lw + w];
    t01[b * 2 * lw + w] = mulmod(x0, y0, m);
    t01[b * 2 * lw + lw + w] = addq(mulmod(x0, y1, m), mulmod(x1, y0, m), m.q);
    t2[b * lw + w] = mulmod(x1, y1, m);
}

// out[b][p][e] = P in[b][p][e] (e <= level), 0 on the special limbs: a
// ciphertext lifted to Q_l U P (pmont: P 2^64 mod q_e)
__global__ __launch_bounds__(kT) void k_scale_ext(u64 *__restrict__ out, const u64 *__restrict__ in, int level, int nE, int N, size_t so,
                                                  size_t si, const u64 *__restrict__ pmont, const ModConst *__restrict__ mods) {
    const int k = blockIdx.x * kT + threadIdx.x, e = blockIdx.y, p = blockIdx.z & 1, b = blockIdx.z >> 1;
    u64 r = 0;
    if (e <= level) {
        const u64 x = in[b * si + ((size_t)p * (level + 1) + e) * N + k], pm = pmont[e];
        r = redc(x * pm, mulhi64(x, pm), mods[e]);
    }
    out[b * so + ((size_t)p * nE + e) * N + k] = r;
}

// Exact residues mod the special primes of centered integers given by
// their limbs mod q_0..q_l (coefficient form).  Garner's mixed-radix digits
//   v_0 = x_0,  v_i = ((x_i - v_0) q_0^-1 - v_1) q_1^-1 ... - v_{i-1}) q_{i-1}^-1 mod q_i,
// give m = sum_i v_i M_i (M_i = q_0 .. q_{i-1}) in [0, Q); m is negative in
// centered form when its digits exceed those of (Q-1)/2 (compared from the
// top); then [m]_p = sum_i v_i [M_i]_p (- [Q]_p).  Table (per level l,
// L1 = l+1): inv[L1][L1] (q_k^-1 mod q_i at [i][k]), mp[L1][nP] ([M_i]_{p_j}
// 2^64, Montgomery), qp[nP] ([Q]_{p_j}), h[L1] (digits of (Q-1)/2).
constexpr int kCrtMax = 32;
__global__ __launch_bounds__(kT) void k_crt_extend(u64 *Xp, const u64 *X, int N, int level, int nP, int pbase,
                                                   const u64 *tab, const ModConst *mods, size_t sxp, size_t sx) {
    const int k = blockIdx.x * kT + threadIdx.x, b = blockIdx.z, L1 = level + 1;
    const u64 *inv = tab, *mp = tab + (size_t)L1 * L1, *qp = mp + (size_t)L1 * nP, *h = qp + nP;
    const u64 *x = X + b * sx + k;
    u64 v[kCrtMax];
#pragma unroll
    for (int i = 0; i < kCrtMax; ++i) {
        if (i < L1) {
            const ModConst mi = mods[i];
            u64 t = x[(size_t)i * N];
            for (int j = 0; j < i; ++j) t = mulmod(subq(t, reduce64(v[j], mi), mi.q), inv[(size_t)i * L1 + j], mi);
            v[i] = t;
        }
    }
    bool neg = false;
    for (int i = level; i >= 0; --i) {
        if (v[i] != h[i]) {
            neg = v[i] > h[i];
            break;
        }
    }
    for (int j = 0; j < nP; ++j) {
        const ModConst mj = mods[pbase + j];
        u64 lo = 0, hi = 0;
#pragma unroll
        for (int i = 0; i < kCrtMax; ++i)
            if (i < L1) mac128(lo, hi, v[i], mp[(size_t)i * nP + j]);
        u64 r = redc_any(lo, hi, mj);
        if (neg) r = subq(r, qp[j], mj.q);
        Xp[b * sxp + (size_t)j * N + k] = r;
    }
}

inline dim3 grid(const fr_ctx *c, int ny, int nz) { return dim3(c->N / kT, ny, nz); }

// P 2^64 mod q_i [L+1], the last ModDown table
inline const u64 *pmont_tab(const fr_ctx *c) {
    const int L1 = c->L + 1, nP = c->nP;
    return c->d_moddown + 2 * nP + (size_t)L1 * nP + 3 * (size_t)L1 + nP + (size_t)L1 * (nP + 1);
}

}  // namespace

namespace frk {

void add(const fr_ctx *c, u64 *out, const u64 *a, const u64 *b, int nlimbs, int npoly, size_t so, size_t sa,
         size_t sb, bool subtract) {
    ProfScope ps(c, K_ELEM, 3.0 * nlimbs * npoly * 8.0 * c->N);
    hipLaunchKernelGGL(k_add, grid(c, nlimbs, npoly), dim3(kT), 0, c->stream, out, a, b, c->N, so, sa, sb, c->d_mod,
                       (int)subtract);
}

void mul_const(const fr_ctx *c, u64 *out, const u64 *a, const u64 *k, const u64 *k_sh, int nlimbs, int npoly,
               size_t so, size_t sa) {
    ProfScope ps(c, K_ELEM, 2.0 * nlimbs * npoly * 8.0 * c->N);
    LimbConsts kc;
    for (int i = 0; i < nlimbs; ++i) {
        kc.v[i] = k[i];
        kc.sh[i] = k_sh[i];
    }
    hipLaunchKernelGGL(k_mul_const, grid(c, nlimbs, npoly), dim3(kT), 0, c->stream, out, a, kc, c->N, so, sa,
                       c->d_mod);
}

void add_const(const fr_ctx *c, u64 *out, const u64 *a, const u64 *k, int nlimbs) {
    ProfScope ps(c, K_ELEM, 2.0 * nlimbs * 8.0 * c->N);
    LimbConsts kc;
    for (int i = 0; i < nlimbs; ++i) kc.v[i] = k[i];
    hipLaunchKernelGGL(k_add_const, grid(c, nlimbs, 1), dim3(kT), 0, c->stream, out, a, kc, c->N, c->d_mod);
}

void mul_pt(const fr_ctx *c, u64 *out, const u64 *a, const u64 *b, int nlimbs, int npoly, size_t so, size_t sa) {
    ProfScope ps(c, K_ELEM, 3.0 * nlimbs * npoly * 8.0 * c->N);
    hipLaunchKernelGGL(k_mul_pt, grid(c, nlimbs, npoly), dim3(kT), 0, c->stream, out, a, b, c->N, so, sa, c->d_mod);
}

void tensor(const fr_ctx *c, u64 *d0, u64 *d1, u64 *d2, const u64 *a0, const u64 *a1, const u64 *b0, const u64 *b1,
            int nlimbs) {
    ProfScope ps(c, K_TENSOR, 7.0 * nlimbs * 8.0 * c->N);
    hipLaunchKernelGGL(k_tensor, grid(c, nlimbs, 1), dim3(kT), 0, c->stream, d0, d1, d2, a0, a1, b0, b1, c->N,
                       c->d_mod);
}

void automorph(const fr_ctx *c, u64 *out, const u64 *in, u64 g, int nlimbs, int npoly, size_t so, size_t si,
               bool accumulate) {
    ProfScope ps(c, K_ELEM, (accumulate ? 3.0 : 2.0) * nlimbs * npoly * 8.0 * c->N);
    hipLaunchKernelGGL(k_automorph, grid(c, nlimbs, npoly), dim3(kT), 0, c->stream, out, in, g, c->N, c->logN, so,
                       si, c->d_mod, (int)accumulate);
}

void mont_scale(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly, size_t poly_stride,
                bool to_mont) {
    ProfScope ps(c, K_ELEM, 2.0 * nlimbs * npoly * 8.0 * c->N);
    hipLaunchKernelGGL(k_mont_scale, grid(c, nlimbs, npoly), dim3(kT), 0, c->stream, data, c->N, poly_stride, map,
                       c->d_mod, (int)to_mont);
}

void modup_digit(const fr_ctx *c, u64 *D, const u64 *x, int level, int t, int batch, size_t sd, size_t sx,
                 const u64 *own, size_t so) {
    const int lo = t * c->alpha, nd = std::min(c->alpha, level + 1 - lo);
    ProfScope ps(c, K_MODUP, (double)batch * (level + 1 + c->nP + (own ? 2 * nd : 0)) * 8.0 * c->N);
    const int nE = level + 1 + c->nP;
    const int ntarget = nE - nd;
    dim3 g(c->N / kT, (ntarget + kTargetsPerThread - 1) / kTargetsPerThread, batch);
    auto kern = nd == 5 ? k_modup<5> : nd == 4 ? k_modup<4> : nd == 1 ? k_modup<1> : k_modup<0>;
    hipLaunchKernelGGL(kern, g, dim3(kT), 0, c->stream, D, x, c->N, lo, nd, nE, level, c->L + 1,
                       c->d_modup + c->modup_off[level][t], c->d_mod, sd, sx, own, so);
}

void modup_all(const fr_ctx *c, u64 *D, const u64 *x, int level, int batch, size_t sd, size_t sx, const u64 *own,
               size_t so) {
    const int nE = level + 1 + c->nP, ndig = (level + c->alpha) / c->alpha;
    for (int t0 = 0; t0 < ndig; t0 += kMaxDigit) {
        const int nt = std::min(kMaxDigit, ndig - t0);
        ProfScope ps(c, K_MODUP, (double)batch * nt * (level + 1 + c->nP) * 8.0 * c->N);
        ModupTabs mt{};
        int maxt = 0;
        for (int t = t0; t < t0 + nt; ++t) {
            mt.tab[t - t0] = c->d_modup + c->modup_off[level][t];
            maxt = std::max(maxt, nE - std::min(c->alpha, level + 1 - t * c->alpha));
        }
        dim3 g(c->N / kT, (maxt + kTargetsPerThread - 1) / kTargetsPerThread, nt * batch);
        auto kern = c->alpha == 5 ? k_modup_all<5> : c->alpha == 1 ? k_modup_all<1> : k_modup_all<0>;
        hipLaunchKernelGGL(kern, g, dim3(kT), 0, c->stream, D, x, c->N, t0, nt, c->alpha, nE, level, c->L + 1,
                           mt, c->d_mod, sd, sx, own, so);
    }
}

// bytes of one key limb set (the nE limbs a key switch at `level` reads)
static double key_limb_bytes(const fr_ctx *c, int level) {
    double b = 0.0;
    for (int e = 0; e < level + 1 + c->nP; ++e)
        b += (c->klay.packed[e <= level ? e : c->L + 1 + (e - level - 1)] ? 5.0 : 8.0) * c->N;
    return b;
}

void ks_inner(const fr_ctx *c, u64 *U0, u64 *U1, const u64 *D, const unsigned char *ksk, u64 g, int level, bool accumulate,
              int batch, size_t sd, size_t su, const u64 *fold_d, size_t fold_sd, const u64 *rot_c0, size_t c0_sd) {
    const int nE_ = level + 1 + c->nP, nd_ = (level + 1 + c->alpha - 1) / c->alpha;
    // digits and outputs per batch item (and c0 when folded in), the shared key once
    ProfScope ps(c, K_KS,
                 batch * (1.0 * nd_ * nE_ + (accumulate ? 4.0 : 2.0) * nE_ + (rot_c0 ? level + 1.0 : 0.0)) * 8.0 *
                         c->N +
                     2.0 * nd_ * key_limb_bytes(c, level));
    const int nE = level + 1 + c->nP;
    const int ndig = (level + 1 + c->alpha - 1) / c->alpha;
    u64 pinv = 0, pinv_sh = 0;
    if (fold_d) {
        pinv = c->P_inv_q[level];
        pinv_sh = c->P_inv_q_sh[level];
    }
    if (c->tune[FR_TUNE_KS_LDS] && ndig >= 1 && ndig <= 3 && batch > 1) {
        // one tile of outputs for every item: the key read once per tile
        auto kern = ndig == 1 ? k_ks_inner_lds<1> : ndig == 2 ? k_ks_inner_lds<2> : k_ks_inner_lds<3>;
        hipLaunchKernelGGL(kern, dim3(c->N / kT, nE, 1), dim3(kT), 0, c->stream, U0, U1, D, ksk, c->klay, g, c->N,
                           c->logN, nE, level, c->L + 1, c->d_mod, (int)accumulate, sd, su, batch, fold_d, fold_sd,
                           pinv, pinv_sh, rot_c0, c0_sd, pmont_tab(c));
        return;
    }
    auto kern = ndig == 1 ? k_ks_inner<1> : ndig == 2 ? k_ks_inner<2> : ndig == 3 ? k_ks_inner<3> : k_ks_inner<0>;
    hipLaunchKernelGGL(kern, dim3(c->N / kT * batch, nE, 1), dim3(kT), 0, c->stream, U0, U1, D, ksk, c->klay, g, c->N,
                       c->logN, nE, level, c->L + 1, ndig, c->d_mod, (int)accumulate, sd, su, batch, fold_d, fold_sd,
                       pinv, pinv_sh, rot_c0, c0_sd, pmont_tab(c));
}

bool ks_inner_multi_ok(const fr_ctx *c, int level) {
    const int ndig = (level + 1 + c->alpha - 1) / c->alpha;
    return ndig >= 1 && ndig <= 3;
}

void ks_inner_multi(const fr_ctx *c, u64 *U, size_t ub, const u64 *D, const unsigned char *const *ksk, const u64 *g,
                    int nrot, int level, int batch, size_t sd, size_t su, const u64 *c0, size_t c0_sd) {
    const int nE = level + 1 + c->nP, ndig = (level + 1 + c->alpha - 1) / c->alpha;
    const u64 twoN = 2ull * (u64)c->N;
    for (int r0 = 0; r0 < nrot; r0 += kMultiRot) {
        const int nr = std::min(kMultiRot, nrot - r0);
        MultiKeys mk{};
        for (int b = 0; b < nr; ++b) {
            mk.ksk[b] = ksk[r0 + b];
            // g^-1 mod 2N (g odd): Newton's iteration for the inverse mod a power of two
            u64 x = g[r0 + b];
            for (int it = 0; it < 6; ++it) x *= 2 - g[r0 + b] * x;
            mk.ginv[b] = x & (twoN - 1);
        }
        // per item: the digit set and c0 once, then per rotation its key and both outputs
        ProfScope ps(c, K_KS,
                     batch * (1.0 * ndig * nE + (level + 1.0) + nr * 2.0 * nE) * 8.0 * c->N +
                         nr * 2.0 * ndig * key_limb_bytes(c, level));
        auto kern = ndig == 1 ? k_ks_inner_multi<1> : ndig == 2 ? k_ks_inner_multi<2> : k_ks_inner_multi<3>;
        hipLaunchKernelGGL(kern, dim3(c->N / kT * batch, nE, 1), dim3(kT), 0, c->stream, U + r0 * ub, ub, D, mk, nr,
                           c->klay, c->N, c->logN, nE, level, c->L + 1, c->d_mod, sd, su, batch, c0, c0_sd,
                           pmont_tab(c));
    }
}

void scale_ext(const fr_ctx *c, u64 *out, const u64 *in, int level, int nb, size_t so, size_t si) {
    const int nE = level + 1 + c->nP;
    ProfScope ps(c, K_ELEM, nb * 2.0 * (level + 1 + nE) * 8.0 * c->N);
    hipLaunchKernelGGL(k_scale_ext, grid(c, nE, 2 * nb), dim3(kT), 0, c->stream, out, in, level, nE, c->N, so, si,
                       pmont_tab(c), c->d_mod);
}

void tensor_sum(const fr_ctx *c, u64 *t01, u64 *t2, int nl, int n, const u64 *const *a, const u64 *const *b) {
    for (int p0 = 0; p0 < n; p0 += kPairs) {
        const int np = std::min(kPairs, n - p0);
        PairPtrs pp{};
        for (int p = 0; p < np; ++p) {
            pp.a[p] = a[p0 + p];
            pp.b[p] = b[p0 + p];
        }
        ProfScope ps(c, K_TENSOR, (4.0 * np + (p0 > 0 ? 6.0 : 3.0)) * nl * 8.0 * c->N);
        hipLaunchKernelGGL(k_tensor_sum, grid(c, nl, 1), dim3(kT), 0, c->stream, t01, t2, pp, np, nl, c->N, c->d_mod,
                           (int)(p0 > 0));
    }
}

int ks_inner_sum_chunk(const fr_ctx *c, int level) {
    const int ndig = (level + c->alpha) / c->alpha;
    return std::max(1, std::min(kGiant, 64 / ndig));
}

void ks_inner_sum(const fr_ctx *c, u64 *U0, u64 *U1, const u64 *D, const unsigned char *const *ksk, const u64 *g, int nj,
                  size_t sdj, int level, bool accumulate, int batch, size_t sd, size_t su) {
    const int nE = level + 1 + c->nP, ndig = (level + c->alpha) / c->alpha;
    GiantKeys gk{};
    for (int j = 0; j < nj; ++j) {
        gk.ksk[j] = ksk[j];
        gk.g[j] = g[j];
    }
    ProfScope ps(c, K_KS,
                 batch * ((double)nj * ndig * nE + (accumulate ? 4.0 : 2.0) * nE) * 8.0 * c->N +
                     2.0 * nj * ndig * key_limb_bytes(c, level));
    if (c->tune[FR_TUNE_KS_LDS] && ndig >= 1 && ndig <= 3) {
        auto kern = ndig == 1 ? k_ks_inner_sum_lds<1> : ndig == 2 ? k_ks_inner_sum_lds<2> : k_ks_inner_sum_lds<3>;
        hipLaunchKernelGGL(kern, dim3(c->N / kT * batch, nE, 1), dim3(kT), 0, c->stream, U0, U1, D, gk, c->klay, nj,
                           sdj, c->N, c->logN, nE, level, c->L + 1, c->d_mod, (int)accumulate, sd, su, batch);
        return;
    }
    auto kern = ndig == 1   ? k_ks_inner_sum<1>
                : ndig == 2 ? k_ks_inner_sum<2>
                : ndig == 3 ? k_ks_inner_sum<3>
                            : k_ks_inner_sum<0>;
    hipLaunchKernelGGL(kern, dim3(c->N / kT * batch, nE, 1), dim3(kT), 0, c->stream, U0, U1, D, gk, c->klay, nj, sdj,
                       c->N, c->logN, nE, level, c->L + 1, ndig, c->d_mod, (int)accumulate, sd, su, batch);
}

void automorph_sum(const fr_ctx *c, u64 *out, const u64 *in, const u64 *g, int nj, int nlimbs, int nb, size_t sob,
                   size_t sij, size_t sib, int level, bool accumulate) {
    for (int j0 = 0; j0 < nj; j0 += kGiant) {
        const int n = std::min(kGiant, nj - j0);
        GiantKeys gk{};
        for (int j = 0; j < n; ++j) gk.g[j] = g[j0 + j];
        const bool acc = accumulate || j0 > 0;
        ProfScope ps(c, K_ELEM, (n + (acc ? 2.0 : 1.0)) * nlimbs * nb * 8.0 * c->N);
        hipLaunchKernelGGL(k_automorph_sum, grid(c, nlimbs, nb), dim3(kT), 0, c->stream, out, in + j0 * sij, gk, n,
                           c->N, c->logN, sob, sij, sib, c->d_mod, level < 0 ? nlimbs : level, c->L + 1, (int)acc);
    }
}

void relin_rescale_prep(const fr_ctx *c, u64 *Z, const u64 *Xu, const u64 *Xd, int level, int npoly, size_t sz,
                        size_t sxu, size_t sxd, bool no_d) {
    ProfScope ps(c, K_MODDOWN, npoly * (2.0 + c->nP + 1.0 * level) * 8.0 * c->N);
    dim3 g(c->N / kT, (level + kFbcTargets - 1) / kFbcTargets, npoly);
    auto kern = c->nP == 5 ? k_relin_rescale_prep<5> : c->nP == 1 ? k_relin_rescale_prep<1> : k_relin_rescale_prep<0>;
    hipLaunchKernelGGL(kern, g, dim3(kT), 0, c->stream, Z, Xu, Xd, c->N, level, c->nP, c->L + 1,
                       c->L + 1, c->d_moddown, c->d_mod, sz, sxu, sxd, (int)no_d, c->d_pbig);
}

void fold_top(const fr_ctx *c, u64 *U, const u64 *d, int level, int npoly, size_t su, size_t sd) {
    hipLaunchKernelGGL(k_fold_top, dim3(c->N / kT, 1, npoly), dim3(kT), 0, c->stream, U, d, c->N, level,
                       c->P_inv_q[level], c->P_inv_q_sh[level], c->d_mod, su, sd);
}
void moddown_fbc(const fr_ctx *c, u64 *V, const u64 *Upc, int level, int npoly) {
    ProfScope ps(c, K_MODDOWN, npoly * (1.0 * c->nP + 1.0 * (level + 1)) * 8.0 * c->N);
    dim3 g(c->N / kT, (level + 1 + kFbcTargets - 1) / kFbcTargets, npoly);
    auto kern = c->nP == 5 ? k_moddown_fbc<5> : c->nP == 1 ? k_moddown_fbc<1> : k_moddown_fbc<0>;
    hipLaunchKernelGGL(kern, g, dim3(kT), 0, c->stream, V, Upc, c->N, level, c->nP, c->L + 1, c->L + 1,
                       c->d_moddown, c->d_mod, (size_t)(level + 1) * c->N, (size_t)c->nP * c->N, c->d_pbig);
}

void moddown_finish(const fr_ctx *c, u64 *out, const u64 *U, const u64 *V, int level, int npoly, size_t so,
                    size_t su, size_t sv, bool accumulate) {
    ProfScope ps(c, K_ELEM, (accumulate ? 4.0 : 3.0) * (level + 1) * npoly * 8.0 * c->N);
    const u64 *pinv = c->d_moddown + 2 * c->nP + (size_t)(c->L + 1) * c->nP;
    const u64 *pinv_sh = pinv + (c->L + 1);
    hipLaunchKernelGGL(k_moddown_finish, grid(c, level + 1, npoly), dim3(kT), 0, c->stream, out, U, V, c->N, pinv,
                       pinv_sh, c->d_mod, so, su, sv, (int)accumulate);
}

void rescale_prep(const fr_ctx *c, u64 *Y, const u64 *xtop, int level, int npoly, size_t sy, size_t sx) {
    ProfScope ps(c, K_RESCALE, (1.0 + level) * npoly * 8.0 * c->N);
    hipLaunchKernelGGL(k_rescale_prep, grid(c, level, npoly), dim3(kT), 0, c->stream, Y, xtop, c->N, level, sy, sx,
                       c->d_mod);
}

void rescale_finish(const fr_ctx *c, u64 *out, const u64 *in, const u64 *Y, int level, int npoly, size_t so,
                    size_t si, size_t sy) {
    ProfScope ps(c, K_RESCALE, 3.0 * level * npoly * 8.0 * c->N);
    const u64 *qinv = c->d_rescale + (size_t)level * (c->L + 1) * 2;
    const u64 *qinv_sh = qinv + (c->L + 1);
    hipLaunchKernelGGL(k_rescale_finish, grid(c, level, npoly), dim3(kT), 0, c->stream, out, in, Y, c->N, qinv,
                       qinv_sh, c->d_mod, so, si, sy);
}

template <int NJ>
static void bsgs_mac_nj(const fr_ctx *c, u64 *P, size_t pq, const u64 *const *baby, int nq, int n1,
                        const unsigned char *const *diag, size_t dstride, const DbLayout &lay, int ell, int level,
                        int baby_level, int lq, int pofs) {
    double dbytes = 0.0;  // bytes of the limbs read per diagonal
    for (int m = 0; m <= level; ++m) dbytes += (lay.packed[m] ? 5.0 : 8.0) * c->N;
    const int n2 = (ell + n1 - 1) / n1;
    for (int q0 = 0; q0 < nq; q0 += kMacQ) {
        const int qn = std::min(kMacQ, nq - q0);
        int ngroups = 0;  // distinct diagonal groups read by this launch
        for (int qq = 0; qq < qn; ++qq) ngroups += qq == 0 || diag[q0 + qq] != diag[q0 + qq - 1];
        for (int j0 = 0; j0 < n2; j0 += NJ) {
            const int nj = std::min(NJ, n2 - j0);
            for (int i0 = 0; i0 < n1; i0 += 32) {
                const int nb = std::min(32, n1 - i0);
                BabyPtrs bp{};
                for (int qq = 0; qq < qn; ++qq) {
                    bp.diag[qq] = diag[q0 + qq];
                    for (int ii = 0; ii < nb; ++ii) bp.p[qq][ii] = baby[(size_t)(q0 + qq) * n1 + i0 + ii];
                }
                long long used = 0;  // diagonal plaintexts of one group this launch reads
                for (int jj = 0; jj < nj; ++jj)
                    for (int ii = 0; ii < nb; ++ii) used += ((j0 + jj) * n1 + i0 + ii < ell);
                ProfScope ps(c, K_MAC,
                             dbytes * ngroups * used +
                                 8.0 * c->N * (level + 1) * qn * (2.0 * nb + (i0 > 0 ? 4.0 : 2.0) * nj));
                // every (j, i) of the tile inside the matrix: no per-term guards
                const bool full = nj == NJ && (j0 + NJ - 1) * n1 + i0 + nb - 1 < ell;
                // the packed and the 64-bit limbs go to launches of their own,
                // so that each compiles to its own register budget; grid.y
                // walks the set bits of the launch's limb mask
                for (int pk = 1; pk >= 0; --pk) {
                    unsigned sel = 0;
                    int nsel = 0;
                    for (int m = 0; m <= level; ++m)
                        if ((lay.packed[m] != 0) == (pk != 0)) sel |= 1u << m, ++nsel;
                    if (!nsel) continue;
                    auto kern = pk ? (full ? k_bsgs_mac3<NJ, true, true> : k_bsgs_mac3<NJ, false, true>)
                                   : (full ? k_bsgs_mac3<NJ, true, false> : k_bsgs_mac3<NJ, false, false>);
                    hipLaunchKernelGGL(kern, dim3(c->N / (kT / 2) * qn, nsel, 1), dim3(kT), 0, c->stream, P + q0 * pq,
                                       pq, bp, qn, nb, i0, n1, j0, nj, ell, dstride, lay, baby_level, level, c->N,
                                       c->d_mod, (int)(i0 > 0), lq, pofs, sel);
                }
            }
        }
    }
}

bool bsgs_ksmac_ok(const fr_ctx *c, int level, int n1, int ell, const DbLayout &lay) {
    const int nE = level + 1 + c->nP, ndig = (level + c->alpha) / c->alpha;
    if (n1 < 2 || n1 > 32 || ell != 16 * n1 || ndig < 1 || ndig > 3 || c->N < kT) return false;
    for (int m = 0; m < nE; ++m) {
        const int gm = m <= level ? m : c->L + 1 + (m - level - 1);
        if ((lay.packed[m] != 0) != (c->klay.packed[gm] != 0)) return false;
    }
    return true;
}

template <int ND>
static void bsgs_ksmac_nd(const fr_ctx *c, u64 *P, size_t pq, int nq, int n1,
                          const unsigned char *const *diag, size_t dstride, const DbLayout &lay, const u64 *D,
                          size_t sd, const u64 *C, size_t sc, const unsigned char *const *ksk, const u64 *g,
                          int level) {
    const int nE = level + 1 + c->nP;
    double dbytes = 0.0;  // bytes of one diagonal's limbs
    for (int m = 0; m < nE; ++m) dbytes += (lay.packed[m] ? 5.0 : 8.0) * c->N;
    for (int q0 = 0; q0 < nq; q0 += kMacQ) {
        const int qn = std::min(kMacQ, nq - q0);
        KsMacSrc ks{};
        int ngroups = 0;
        for (int qq = 0; qq < qn; ++qq) {
            ks.diag[qq] = diag[q0 + qq];
            ngroups += qq == 0 || diag[q0 + qq] != diag[q0 + qq - 1];
        }
        for (int i = 1; i < n1; ++i) ks.ksk[i] = ksk[i], ks.g[i] = g[i];
        ks.ksk[0] = ks.ksk[1];
        // algorithmic bytes: every diagonal of the groups once, each query's
        // digit set, the query and the outputs once, every key once
        ProfScope ps(c, K_MAC,
                     dbytes * ngroups * 16.0 * n1 +
                         8.0 * c->N * qn * (ND * nE + 2.0 * (level + 1.0) + 2.0 * 16 * nE) +
                         (n1 - 1) * 2.0 * ND * key_limb_bytes(c, level));
        for (int pk = 1; pk >= 0; --pk) {
            unsigned sel = 0;
            int nsel = 0;
            for (int m = 0; m < nE; ++m)
                if ((lay.packed[m] != 0) == (pk != 0)) sel |= 1u << m, ++nsel;
            if (!nsel) continue;
            auto kern = pk ? k_bsgs_ksmac<16, true, ND> : k_bsgs_ksmac<16, false, ND>;
            hipLaunchKernelGGL(kern, dim3(c->N / (kT / 2) * qn, nsel, 1), dim3(kT), 0, c->stream, P + q0 * pq, pq, ks,
                               qn, n1, n1, dstride, lay, c->klay, D + q0 * sd, sd, C + q0 * sc, sc, nE, level,
                               c->L - level, c->logN, c->N, c->d_mod, pmont_tab(c), sel);
        }
    }
}

void bsgs_ksmac(const fr_ctx *c, u64 *P, size_t pq, int nq, int n1,
                const unsigned char *const *diag, size_t dstride, const DbLayout &lay, const u64 *D, size_t sd,
                const u64 *C, size_t sc, const unsigned char *const *ksk, const u64 *g, int level) {
    const int ndig = (level + c->alpha) / c->alpha;
    auto f = ndig == 1 ? bsgs_ksmac_nd<1> : ndig == 2 ? bsgs_ksmac_nd<2> : bsgs_ksmac_nd<3>;
    f(c, P, pq, nq, n1, diag, dstride, lay, D, sd, C, sc, ksk, g, level);
}

// giant steps per thread: 16, or the smallest power of two covering n2
void bsgs_mac(const fr_ctx *c, u64 *P, size_t pq, const u64 *const *baby, int nq, int n1,
              const unsigned char *const *diag, size_t dstride, const DbLayout &lay, int ell, int level,
              int baby_level, int lq, int pofs) {
    const int n2 = (ell + n1 - 1) / n1;
    if (n2 > 8)
        bsgs_mac_nj<16>(c, P, pq, baby, nq, n1, diag, dstride, lay, ell, level, baby_level, lq, pofs);
    else if (n2 > 4)
        bsgs_mac_nj<8>(c, P, pq, baby, nq, n1, diag, dstride, lay, ell, level, baby_level, lq, pofs);
    else if (n2 > 2)
        bsgs_mac_nj<4>(c, P, pq, baby, nq, n1, diag, dstride, lay, ell, level, baby_level, lq, pofs);
    else if (n2 > 1)
        bsgs_mac_nj<2>(c, P, pq, baby, nq, n1, diag, dstride, lay, ell, level, baby_level, lq, pofs);
    else
        bsgs_mac_nj<1>(c, P, pq, baby, nq, n1, diag, dstride, lay, ell, level, baby_level, lq, pofs);
}

void db_pack(const fr_ctx *c, unsigned char *dst, size_t dstride, const DbLayout &lay, const u64 *src, int nl, int nd) {
    if (nd <= 0) return;
    hipLaunchKernelGGL(k_db_pack, grid(c, nl, nd), dim3(kT), 0, c->stream, dst, dstride, lay, src, nl, c->N);
}

void db_unpack(const fr_ctx *c, u64 *dst, const unsigned char *src, size_t sstride, const DbLayout &lay, int nl,
               int nd) {
    if (nd <= 0) return;
    hipLaunchKernelGGL(k_db_unpack, grid(c, nl, nd), dim3(kT), 0, c->stream, dst, src, sstride, lay, nl, c->N);
}

void key_pack(const fr_ctx *c, unsigned char *dst, const u64 *src, int nb) {
    hipLaunchKernelGGL(k_key_pack, grid(c, c->nmod, nb), dim3(kT), 0, c->stream, dst, c->klay, src, c->nmod, c->N);
}

void key_unpack(const fr_ctx *c, u64 *dst, const unsigned char *src, int nb) {
    hipLaunchKernelGGL(k_key_unpack, grid(c, c->nmod, nb), dim3(kT), 0, c->stream, dst, c->klay, src, c->nmod, c->N);
}

void moddown_rot(const fr_ctx *c, u64 *const *out, const u64 *U, const u64 *V, const u64 *const *in, u64 g,
                 int level, int nitems) {
    const u64 *pinv = c->d_moddown + 2 * c->nP + (size_t)(c->L + 1) * c->nP;
    const u64 *pinv_sh = pinv + (c->L + 1);
    const int nE = level + 1 + c->nP;
    const size_t lw = (size_t)(level + 1) * c->N;
    for (int b0 = 0; b0 < nitems; b0 += kBatch) {
        const int nb = std::min(kBatch, nitems - b0);
        RotItems it{};
        for (int b = 0; b < nb; ++b) {
            it.out[b] = out[b0 + b];
            it.in[b] = in[b0 + b];
        }
        ProfScope ps(c, K_ELEM, nb * 7.0 * (level + 1) * 8.0 * c->N);
        hipLaunchKernelGGL(k_moddown_rot, grid(c, level + 1, 2 * nb), dim3(kT), 0, c->stream, it,
                           U + (size_t)b0 * 2 * nE * c->N, V + (size_t)b0 * 2 * lw, g, c->N, c->logN, level + 1,
                           pinv, pinv_sh, c->d_mod, (size_t)nE * c->N);
    }
}


void scalar_batch(const fr_ctx *c, u64 *out, int nl, int B, const ScalarItem *items) {
    for (int b0 = 0; b0 < B; b0 += kBatch) {
        const int nb = std::min(kBatch, B - b0);
        size_t most = 0;
        for (int b = 0; b < nb; ++b) most = std::max(most, items[b0 + b].src.size());
        for (size_t t0 = 0; t0 == 0 || t0 < most; t0 += kTerms) {
            ScalarBatch sb{};
            sb.accumulate = t0 > 0;
            int terms = 0;
            for (int b = 0; b < nb; ++b) {
                const ScalarItem &it = items[b0 + b];
                const int nt = (int)std::min<size_t>(kTerms, it.src.size() > t0 ? it.src.size() - t0 : 0);
                sb.nterms[b] = nt;
                for (int t = 0; t < nt; ++t) {
                    sb.src[b][t] = it.src[t0 + t];
                    sb.k[b][t] = it.k[t0 + t];
                    sb.src_lp1[b][t] = it.lp1[t0 + t];
                }
                terms += nt;
            }
            ProfScope ps(c, K_ELEM, (terms + nb * (sb.accumulate ? 2.0 : 1.0)) * 2.0 * nl * 8.0 * c->N);
            hipLaunchKernelGGL(k_scalar_batch, grid(c, 2 * nl, nb), dim3(kT), 0, c->stream,
                               out + (size_t)b0 * 2 * nl * c->N, sb, nl, c->N, c->d_mod);
        }
    }
}

bool scalar_mat(const fr_ctx *c, u64 *out, int nl, int nb, int nq, const u64 *const *src, const int *lp1, int ns,
                const long long *K, size_t ob, size_t oq) {
    if (nb > kMatB || ns > kMatS || nq > kMatQ || nb < 1 || ns < 1) return false;
    ScalarMat sm{};
    sm.ns = ns;
    sm.nb = nb;
    for (int s = 0; s < ns; ++s) {
        sm.lp1[s] = lp1[s];
        for (int q = 0; q < nq; ++q) sm.src[q][s] = src[(size_t)q * ns + s];
    }
    for (int b = 0; b < nb; ++b)
        for (int s = 0; s < ns; ++s) {
            sm.k[b][s] = K[(size_t)b * ns + s];
            if (sm.k[b][s]) sm.nz[b] |= 1u << s;
        }
    ProfScope ps(c, K_ELEM, (double)nq * (ns + nb) * 2.0 * nl * 8.0 * c->N);
    hipLaunchKernelGGL(k_scalar_mat, grid(c, 2 * nl, nq), dim3(kT), 0, c->stream, out, ob, oq, sm, nl, c->N,
                       c->d_mod);
    return true;
}

void add_const_batch(const fr_ctx *c, u64 *data, int nl, int B, const long long *v, size_t item) {
    for (int b0 = 0; b0 < B; b0 += kBatch) {
        const int nb = std::min(kBatch, B - b0);
        ConstBatch cb{};
        for (int b = 0; b < nb; ++b) cb.v[b] = v[b0 + b];
        ProfScope ps(c, K_ELEM, nb * 2.0 * nl * 8.0 * c->N);
        hipLaunchKernelGGL(k_add_const_batch, grid(c, nl, nb), dim3(kT), 0, c->stream, data + b0 * item, cb, nl,
                           c->N, item, c->d_mod);
    }
}

void pair_batch(const fr_ctx *c, int nl, int B, const u64 *const *a, const u64 *const *b, u64 *const *out,
                const long long *cst, const int *op) {
    for (int b0 = 0; b0 < B; b0 += kBatch) {
        const int nb = std::min(kBatch, B - b0);
        PairBatch pb{};
        for (int t = 0; t < nb; ++t) {
            pb.a[t] = a[b0 + t];
            pb.b[t] = b[b0 + t];
            pb.out[t] = out[b0 + t];
            pb.cst[t] = cst[b0 + t];
            pb.op[t] = op[b0 + t];
        }
        ProfScope ps(c, K_ELEM, nb * 6.0 * nl * 8.0 * c->N);
        hipLaunchKernelGGL(k_pair_batch, grid(c, 2 * nl, nb), dim3(kT), 0, c->stream, pb, nl, c->N, c->d_mod);
    }
}

void tensor_batch(const fr_ctx *c, u64 *t01, u64 *t2, int nl, int B, const u64 *const *a, const u64 *const *b) {
    for (int b0 = 0; b0 < B; b0 += kBatch) {
        const int nb = std::min(kBatch, B - b0);
        TensorBatch tb{};
        for (int t = 0; t < nb; ++t) {
            tb.a[t] = a[b0 + t];
            tb.b[t] = b[b0 + t];
        }
        ProfScope ps(c, K_TENSOR, nb * 7.0 * nl * 8.0 * c->N);
        const size_t lw = (size_t)nl * c->N;
        hipLaunchKernelGGL(k_tensor_batch, grid(c, nl, nb), dim3(kT), 0, c->stream, t01 + (size_t)b0 * 2 * lw,
                           t2 + (size_t)b0 * lw, tb, nl, c->N, c->d_mod);
    }
}

void key_combine(const fr_ctx *c, u64 *b, const u64 *a, const u64 *e, const u64 *s_mont, const u64 *sp, int dlo,
                 int dhi, int nlimbs) {
    LimbConsts pm;
    for (int i = 0; i < nlimbs && i < FR_MAXMOD; ++i) {
        pm.v[i] = i <= c->L ? c->P_mod_q[i] : 0;
        pm.sh[i] = i <= c->L ? c->P_mod_q_sh[i] : 0;
    }
    hipLaunchKernelGGL(k_key_combine, grid(c, nlimbs, 1), dim3(kT), 0, c->stream, b, a, e, s_mont, sp, pm, dlo, dhi,
                       c->N, c->d_mod);
}

void encrypt_combine(const fr_ctx *c, u64 *c0, u64 *c1, const u64 *v, const u64 *e0, const u64 *e1, const u64 *msg,
                     const u64 *pkb, const u64 *pka, int nlimbs) {
    hipLaunchKernelGGL(k_encrypt_combine, grid(c, nlimbs, 1), dim3(kT), 0, c->stream, c0, c1, v, e0, e1, msg, pkb,
                       pka, c->N, c->d_mod);
}

void decrypt_combine(const fr_ctx *c, u64 *out, const u64 *c0, const u64 *c1, const u64 *s_mont, int nlimbs) {
    hipLaunchKernelGGL(k_decrypt_combine, grid(c, nlimbs, 1), dim3(kT), 0, c->stream, out, c0, c1, s_mont, c->N,
                       c->d_mod);
}

int crt_extend(fr_ctx *c, u64 *Xp, const u64 *X, int level, int npoly, size_t sxp, size_t sx) {
    const int L1 = level + 1, nP = c->nP;
    if (L1 > kCrtMax) return fr_fail(FR_EINVAL, "crt_extend: %d limbs exceed %d", L1, kCrtMax);
    std::vector<u64> t((size_t)L1 * L1 + (size_t)L1 * nP + nP + L1, 0);
    u64 *inv = t.data(), *mp = inv + (size_t)L1 * L1, *qp = mp + (size_t)L1 * nP, *h = qp + nP;
    for (int i = 0; i < L1; ++i)
        for (int j = 0; j < i; ++j) inv[(size_t)i * L1 + j] = frh::invmod_h(c->mod[j] % c->mod[i], c->mod[i]);
    for (int j = 0; j < nP; ++j) {
        const u64 p = c->mod[c->L + 1 + j], r64 = (0 - p) % p;
        u64 M = 1 % p;
        for (int i = 0; i < L1; ++i) {
            mp[(size_t)i * nP + j] = frh::mulmod_h(M, r64, p);
            M = frh::mulmod_h(M, c->mod[i] % p, p);
        }
        qp[j] = M;
    }
    // (Q-1)/2 digit by digit from the top: Q-1 has the digits q_i - 1
    u64 r = 0;
    for (int i = level; i >= 0; --i) {
        const u64 cur = (c->mod[i] - 1) + r * c->mod[i];
        h[i] = cur >> 1;
        r = cur & 1;
    }
    u64 *d = (u64 *)c->arena.get(t.size() * 8);
    if (!d) return fr_fail(FR_ENOMEM, "crt_extend: scratch");
    if (hipMemcpyAsync(d, t.data(), t.size() * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return fr_fail(FR_EHIP, "crt_extend: table upload");
    hipLaunchKernelGGL(k_crt_extend, dim3(c->N / kT, 1, npoly), dim3(kT), 0, c->stream, Xp, X, c->N, level, nP,
                       c->L + 1, d, c->d_mod, sxp, sx);
    // the table lives in host memory until the copy has run
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fr_fail(FR_EHIP, "crt_extend: synchronize");
    return FR_OK;
}

}  // namespace frk
