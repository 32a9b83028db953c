// kernels_ntt.hip -- negacyclic NTT / inverse NTT on uint64 limbs (gfx950).
//
// Forward transform: Cooley-Tukey with the 2N-th root psi merged into the
// twiddles (tw[k] = psi^brv(k)), natural order in, bit-reversed order out.
// Inverse: Gentleman-Sande with itw[k] = psi^-brv(k), then N^-1.
//
// N = R1 * C with R1 = 2^floor(logN/2).  Stages whose butterfly distance is
// a multiple of C act on the R1 words of one "column" (stride C); the other
// stages act inside contiguous blocks of C words.  Each pass stages a tile
// of up to 4096 words (32 KiB) in LDS: several adjacent columns, so that the
// strided loads of the column pass still fill 128-byte lines, or several
// contiguous blocks for the row pass.
#include "fr_core.h"

namespace {

constexpr int kTile = 4096;
constexpr int kThreads = 256;

struct NttLaunch {
    u64 *data;
    size_t poly_stride;
    const u64 *src;          // first pass reads here when set (out-of-place)
    size_t src_poly_stride;
    int N, logN, s1;
    LimbMap map;
    const u64 *tw, *tw_sh;
    const ulonglong2 *tw2;   // (twiddle, Shoup companion) pairs, same indexing
    const ModConst *mods;
    // rescale fused into a forward transform (radix-16 kernels only):
    // pre_top >= 0: the first pass reads src as ONE limb per polynomial and
    // maps x to the centered residue of x mod q_pre_top in the target limb;
    // epi_out != nullptr: the last pass writes epi_out = (epi_in - y) qinv
    // (+ epi_out if epi_acc) instead of y (rescale or ModDown finish)
    int pre_top;
    int epi_acc;
    // qinv2 != nullptr: epi_out = (epi_in2 + (epi_in - y) qinv) qinv2, without
    // the epi_in2 term when it is null (ModDown merged with a rescale)
    const u64 *epi_in2;
    size_t epi_in2_stride;
    const u64 *qinv2, *qinv2_sh;
    u64 *epi_out;
    const u64 *epi_in;
    size_t epi_out_stride, epi_in_stride;
    const u64 *qinv, *qinv_sh;
    // ModUp digit sets (own_alpha > 0): polynomial z is digit z % own_ndig,
    // whose own limbs [t alpha, min(t alpha + alpha, own_nlq)) are already in
    // evaluation form; the forward passes leave them untouched
    int own_alpha, own_ndig, own_nlq;
};

__device__ __forceinline__ bool own_skip(const NttLaunch &a, int s, int poly) {
    if (!a.own_alpha) return false;
    const int lo = (poly % a.own_ndig) * a.own_alpha;
    return s >= lo && s < lo + a.own_alpha && s < a.own_nlq;
}

__global__ __launch_bounds__(kThreads) void k_fwd_cols(NttLaunch a) {
    __shared__ u64 tile[kTile];
    const int lr = a.s1, lc = a.logN - a.s1;
    const int R1 = 1 << lr, C = 1 << lc;
    const int lcols = min(12 - lr, lc), COLS = 1 << lcols;
    const int total = R1 * COLS;
    const int s = a.map.storage(blockIdx.y);
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q;
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * a.N;
    const u64 *tw = a.tw + (size_t)mi * a.N, *twsh = a.tw_sh + (size_t)mi * a.N;
    const int c0 = blockIdx.x * COLS;
    const u64 *xs = a.src ? a.src + blockIdx.z * a.src_poly_stride + (size_t)s * a.N : x;
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        int r = idx >> lcols, c = idx & (COLS - 1);
        tile[idx] = xs[c0 + c + ((size_t)r << lc)];
    }
    __syncthreads();
    for (int st = 0; st < lr; ++st) {
        const int m = 1 << st, ltp = lr - st - 1, tp = 1 << ltp;
        for (int b = threadIdx.x; b < (total >> 1); b += kThreads) {
            const int c = b & (COLS - 1), bb = b >> lcols;
            const int i = bb >> ltp, jj = bb & (tp - 1);
            const int r = (i << (ltp + 1)) + jj;
            const u64 w = tw[m + i], wsh = twsh[m + i];
            const int i0 = (r << lcols) + c, i1 = ((r + tp) << lcols) + c;
            const u64 U = tile[i0];
            const u64 V = shoup(tile[i1], w, wsh, q);
            tile[i0] = addq(U, V, q);
            tile[i1] = subq(U, V, q);
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        int r = idx >> lcols, c = idx & (COLS - 1);
        x[c0 + c + ((size_t)r << lc)] = tile[idx];
    }
}

__global__ __launch_bounds__(kThreads) void k_fwd_rows(NttLaunch a) {
    __shared__ u64 tile[kTile];
    const int lr = a.s1, lc = a.logN - a.s1;
    const int R1 = 1 << lr, C = 1 << lc;
    const int lblks = min(12 - lc, lr), BLKS = 1 << lblks;
    const int total = BLKS * C;
    const int s = a.map.storage(blockIdx.y);
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q;
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * a.N + (size_t)blockIdx.x * total;
    const u64 *tw = a.tw + (size_t)mi * a.N, *twsh = a.tw_sh + (size_t)mi * a.N;
    const int b0 = blockIdx.x * BLKS;
    (void)R1;
    for (int idx = threadIdx.x; idx < total; idx += kThreads) tile[idx] = x[idx];
    __syncthreads();
    for (int st = lr; st < a.logN; ++st) {
        const int m = 1 << st, lt = a.logN - st - 1, t = 1 << lt;
        for (int b = threadIdx.x; b < (total >> 1); b += kThreads) {
            const int blk = b >> (lc - 1), u2 = b & ((C >> 1) - 1);
            const int il = u2 >> lt, jj = u2 & (t - 1);
            const int u = (il << (lt + 1)) + jj;
            const int i = ((b0 + blk) << (lc - 1 - lt)) + il;
            const u64 w = tw[m + i], wsh = twsh[m + i];
            const int i0 = (blk << lc) + u, i1 = i0 + t;
            const u64 U = tile[i0];
            const u64 V = shoup(tile[i1], w, wsh, q);
            tile[i0] = addq(U, V, q);
            tile[i1] = subq(U, V, q);
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < total; idx += kThreads) x[idx] = tile[idx];
}

__global__ __launch_bounds__(kThreads) void k_inv_rows(NttLaunch a) {
    __shared__ u64 tile[kTile];
    const int lr = a.s1, lc = a.logN - a.s1;
    const int C = 1 << lc;
    const int lblks = min(12 - lc, lr), BLKS = 1 << lblks;
    const int total = BLKS * C;
    const int s = a.map.storage(blockIdx.y);
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q;
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * a.N + (size_t)blockIdx.x * total;
    const u64 *tw = a.tw + (size_t)mi * a.N, *twsh = a.tw_sh + (size_t)mi * a.N;
    const int b0 = blockIdx.x * BLKS;
    const u64 *xs = a.src ? a.src + blockIdx.z * a.src_poly_stride + (size_t)s * a.N + (size_t)blockIdx.x * total : x;
    for (int idx = threadIdx.x; idx < total; idx += kThreads) tile[idx] = xs[idx];
    __syncthreads();
    for (int lt = 0; lt < lc; ++lt) {  // t = 1, 2, .., C/2
        const int t = 1 << lt;
        const int h = a.N >> (lt + 1);
        for (int b = threadIdx.x; b < (total >> 1); b += kThreads) {
            const int blk = b >> (lc - 1), u2 = b & ((C >> 1) - 1);
            const int il = u2 >> lt, jj = u2 & (t - 1);
            const int u = (il << (lt + 1)) + jj;
            const int i = ((b0 + blk) << (lc - 1 - lt)) + il;
            const u64 w = tw[h + i], wsh = twsh[h + i];
            const int i0 = (blk << lc) + u, i1 = i0 + t;
            const u64 U = tile[i0], V = tile[i1];
            tile[i0] = addq(U, V, q);
            tile[i1] = shoup(subq(U, V, q), w, wsh, q);
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < total; idx += kThreads) x[idx] = tile[idx];
}

__global__ __launch_bounds__(kThreads) void k_inv_cols(NttLaunch a) {
    __shared__ u64 tile[kTile];
    const int lr = a.s1, lc = a.logN - a.s1;
    const int R1 = 1 << lr;
    const int lcols = min(12 - lr, lc), COLS = 1 << lcols;
    const int total = R1 * COLS;
    const int s = a.map.storage(blockIdx.y);
    const int mi = a.map.modidx(s);
    const ModConst mc = a.mods[mi];
    const u64 q = mc.q;
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * a.N;
    const u64 *tw = a.tw + (size_t)mi * a.N, *twsh = a.tw_sh + (size_t)mi * a.N;
    const int c0 = blockIdx.x * COLS;
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        int r = idx >> lcols, c = idx & (COLS - 1);
        tile[idx] = x[c0 + c + ((size_t)r << lc)];
    }
    __syncthreads();
    for (int ltp = 0; ltp < lr; ++ltp) {  // t = C t', t' = 1 .. R1/2
        const int tp = 1 << ltp;
        const int h = a.N >> (lc + ltp + 1);
        for (int b = threadIdx.x; b < (total >> 1); b += kThreads) {
            const int c = b & (COLS - 1), bb = b >> lcols;
            const int i = bb >> ltp, jj = bb & (tp - 1);
            const int r = (i << (ltp + 1)) + jj;
            const u64 w = tw[h + i], wsh = twsh[h + i];
            const int i0 = (r << lcols) + c, i1 = ((r + tp) << lcols) + c;
            const u64 U = tile[i0], V = tile[i1];
            tile[i0] = addq(U, V, q);
            tile[i1] = shoup(subq(U, V, q), w, wsh, q);
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        int r = idx >> lcols, c = idx & (COLS - 1);
        x[c0 + c + ((size_t)r << lc)] = shoup(tile[idx], mc.ninv, mc.ninv_sh, q);
    }
}


// ---------------------------------------------------------------------------
// Radix-2^LE register kernels for even logN = 4 LE (N = 2^12, 2^16): every
// 2^(2 LE)-point sub-transform is done by E = 2^LE threads, E coefficients
// each, in two register rounds of LE stages with one LDS transpose between
// them.  Butterflies are Harvey's lazy forms with a truncated Shoup quotient
// (forward values in [0, 8q), inverse in [0, 4q); every prime is below 2^61
// so 8q fits a word); outputs are reduced to [0, q).  Round-1 twiddles of
// the column pass are uniform across the workgroup.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 shoup_lazy(u64 a, u64 w, u64 wp, u64 q) { return a * w - mulhi64(a, wp) * q; }

// 2^64 - q, hidden from the compiler so that a w - h q is formed as
// a w + h (2^64 - q): the second product then accumulates onto the first
__device__ __forceinline__ u64 opaque_neg(u64 q) {
    u64 nq = 0 - q;
    asm("" : "+s"(nq));
    return nq;
}

// a * w - h q with h the high word of a * wp built from the three partial
// products that reach it (the low 32x32 product and the carries out of the
// middle products' low halves are dropped): h is at most 2 below the exact
// quotient estimate, so the result lies in [0, 4q) for any 64-bit a.
__device__ __forceinline__ u64 shoup_lazy4(u64 a, u64 w, u64 wp, u64 nq) {
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), p0 = (u32)wp, p1 = (u32)(wp >> 32);
    const u64 h = (u64)a1 * p1 + __umulhi(a0, p1) + __umulhi(a1, p0);
    return a * w + h * nq;
}

// Forward butterfly.  Large primes: inputs and outputs in [0, 8q), x
// reduced below 4q first.  Small primes (q < 2^46, SMALL): no reduction at
// all, the bound grows by 4q per stage (at most 65q after 16 stages).
template <bool SMALL>
__device__ __forceinline__ void ct_bfly(u64 &X, u64 &Y, u64 w, u64 wp, u64 q, u64 q4, u64 nq) {
    u64 x = X;
    if (!SMALL) x = X >= q4 ? X - q4 : X;
    const u64 t = shoup_lazy4(Y, w, wp, nq);
    X = x + t;
    Y = x - t + q4;
}
// Inverse butterfly.  Large primes: inputs and outputs in [0, 4q).  Small
// primes: the sum is not reduced and M (a multiple of q at least the input
// bound) keeps the difference positive; the bound doubles per stage (below
// q 2^17 after 16 stages).
template <bool SMALL>
__device__ __forceinline__ void gs_bfly(u64 &X, u64 &Y, u64 w, u64 wp, u64 q, u64 q4, u64 nq, u64 M) {
    u64 s = X + Y;
    if (!SMALL) s = s >= q4 ? s - q4 : s;
    const u64 d = X - Y + (SMALL ? M : q4);
    X = s;
    Y = shoup_lazy4(d, w, wp, nq);
}
// primes below this take the reduction-free butterflies
constexpr u64 kSmallQ = 1ull << 46;

// A stage's twiddles are tw[base + (k >> sh)] for its elements k < E.  With
// HOLD all E >> sh of them are fetched before the stage's butterflies and
// the scheduler may not sink the loads back to their uses, so they overlap
// instead of each waiting for the one before (more registers: measured
// worth it only in the plain forward row pass, whose large-stage twiddles
// come from L2).  Without HOLD each is loaded at its use.
#define NTT_STAGE_TW(HOLD, BASE, SH)                                                                     \
    ulonglong2 tws[E];                                                                                    \
    const int tbase_ = (BASE);                                                                            \
    if (HOLD) {                                                                                           \
        _Pragma("unroll") for (int t = 0; t < E; ++t) if (t < (E >> (SH))) tws[t] = tw[tbase_ + t];      \
        __builtin_amdgcn_sched_barrier(0);                                                                \
    }
#define NTT_TW(HOLD, K, SH) ((HOLD) ? tws[(K) >> (SH)] : tw[tbase_ + ((K) >> (SH))])

// LDS layouts of the transposes.  A row tile of R = E^2 words is read both
// as i = u + E k and as i = E u + k (u the lane's index); word i = E r + c of
// the tile of sub-transform `blk` is stored at E (r ^ blk mod E) + (c ^ r),
// which spreads both patterns of a wave evenly over the banks.  The column
// tiles (COLS words per row) are read as rows g + E k and E g + k; row r is
// stored at r ^ ((r >> LE) & 1) so that the second pattern uses both halves
// of the banks.
template <int LE>
__device__ __forceinline__ int rsw(int i, int blk) {
    constexpr int E = 1 << LE;
    const int r = i >> LE, c = i & (E - 1);
    return (((r ^ blk) & (E - 1)) << LE) | (c ^ r);
}
template <int LE>
__device__ __forceinline__ int csw(int row) { return row ^ ((row >> LE) & 1); }

__device__ __forceinline__ u64 red8(u64 x, u64 q) {
    x = x >= 4 * q ? x - 4 * q : x;
    x = x >= 2 * q ? x - 2 * q : x;
    return x >= q ? x - q : x;
}
// canonical forward output: [0, 8q) (large) or [0, 65q) (small)
template <bool SMALL>
__device__ __forceinline__ u64 fwd_final(u64 x, const ModConst &m) {
    return SMALL ? reduce64(x, m) : red8(x, m.q);
}

template <int LE, bool SMALL>
__device__ __forceinline__ void k_fwd_cols2_body(const NttLaunch &a, u64 *tile) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, COLS = kThreads / E;
    const int s = a.map.storage(blockIdx.y);
    if (own_skip(a, s, blockIdx.z)) return;
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * a.N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * a.N;
    const int c = threadIdx.x % COLS, g = threadIdx.x / COLS;
    const int col = blockIdx.x * COLS + c;
    const u64 *xs = a.src ? a.src + blockIdx.z * a.src_poly_stride + (a.pre_top >= 0 ? 0 : (size_t)s * a.N) : x;
    u64 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = xs[col + (size_t)(g + E * k) * R];
    if (a.pre_top >= 0) {  // centered residue of the top limb in this limb
        const u64 qt = a.mods[a.pre_top].q;
        const ModConst mc = a.mods[mi];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            if (v[k] > (qt >> 1)) {
                const u64 neg = reduce64(qt - v[k], mc);
                v[k] = neg ? mc.q - neg : 0;
            } else {
                v[k] = reduce64(v[k], mc);
            }
        }
    }
#pragma unroll
    for (int st = 0; st < LE; ++st) {
        const int half = E >> (st + 1);
        NTT_STAGE_TW(false, 1 << st, LE - st)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(false, k, LE - st);
                ct_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq);
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) tile[csw<LE>(g + E * k) * COLS + c] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = tile[csw<LE>(E * g + k) * COLS + c];
#pragma unroll
    for (int st = LE; st < LR; ++st) {
        const int half = 1 << (LR - st - 1);
        NTT_STAGE_TW(false, (1 << st) + (g << (st - LE)), LR - st)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(false, k, LR - st);
                ct_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq);
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) x[col + (size_t)(E * g + k) * R] = v[k];
}

template <int LE>
__global__ __launch_bounds__(kThreads) void k_fwd_cols2(NttLaunch a) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, COLS = kThreads / E;
    __shared__ u64 tile[R * COLS];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.y))].q;
    if (qb < kSmallQ)
        k_fwd_cols2_body<LE, true>(a, tile);
    else
        k_fwd_cols2_body<LE, false>(a, tile);
}

template <int LE, bool SMALL, bool EPI>
__device__ __forceinline__ void k_fwd_rows2_body(const NttLaunch &a, u64 *tile) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, BLKS = kThreads / E;
    const int s = a.map.storage(blockIdx.z);
    if (own_skip(a, s, blockIdx.y)) return;
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    const ModConst mcq = a.mods[mi];
    u64 *x = a.data + blockIdx.y * a.poly_stride + (size_t)s * a.N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * a.N;
    const int blk = threadIdx.x / E, u0 = threadIdx.x % E;
    const int gb = blockIdx.x * BLKS + blk;
    u64 *xb = x + (size_t)gb * R;
    u64 *tb = tile + blk * R;
    u64 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = xb[u0 + E * k];
    // the epilogue's operands are fetched now, their latency hidden by the
    // butterflies (issued after v, so waiting for v leaves them in flight)
    const size_t w = (size_t)s * a.N + (size_t)gb * R;
    u64 pin[EPI ? E : 1], pin2[EPI ? E : 1];
    if constexpr (EPI) {
        const u64 *in = a.epi_in + blockIdx.y * a.epi_in_stride + w;
#pragma unroll
        for (int k = 0; k < E; ++k) pin[k] = in[u0 + E * k];
        if (a.epi_in2) {
            const u64 *in2 = a.epi_in2 + blockIdx.y * a.epi_in2_stride + w;
#pragma unroll
            for (int k = 0; k < E; ++k) pin2[k] = in2[u0 + E * k];
        }
    }
#pragma unroll
    for (int sl = 0; sl < LE; ++sl) {
        const int half = E >> (sl + 1);
        NTT_STAGE_TW(!EPI, (1 << (LR + sl)) + (gb << sl), LE - sl)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(!EPI, k, LE - sl);
                ct_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq);
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) tb[rsw<LE>(u0 + E * k, blk)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = tb[rsw<LE>(E * u0 + k, blk)];
#pragma unroll
    for (int sl = LE; sl < LR; ++sl) {
        const int half = 1 << (LR - sl - 1);
        NTT_STAGE_TW(!EPI, (1 << (LR + sl)) + (gb << sl) + (u0 << (sl - LE)), LR - sl)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(!EPI, k, LR - sl);
                ct_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq);
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) tb[rsw<LE>(E * u0 + k, blk)] = v[k];
    __syncthreads();
    // rescale / ModDown finish: (in - y) qinv (+ out).  The plain variant
    // keeps the same branch, read directly (it never runs there; kept so both
    // variants compile to the same register budget for the common part)
    if (EPI || a.epi_out) {
        const u64 *in = a.epi_in + blockIdx.y * a.epi_in_stride + w;
        const u64 *in2 = a.epi_in2 ? a.epi_in2 + blockIdx.y * a.epi_in2_stride + w : nullptr;
        auto x_in = [&](int k) { if constexpr (EPI) return pin[k]; else return in[u0 + E * k]; };
        auto x_in2 = [&](int k) { if constexpr (EPI) return pin2[k]; else return in2[u0 + E * k]; };
        u64 *out = a.epi_out + blockIdx.y * a.epi_out_stride + w;
        const u64 qi = a.qinv[mi], qs = a.qinv_sh[mi];
        if (a.qinv2) {
            const u64 q2i = a.qinv2[mi], q2s = a.qinv2_sh[mi];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                u64 r = shoup(subq(x_in(k), fwd_final<SMALL>(tb[rsw<LE>(u0 + E * k, blk)], mcq), q), qi, qs, q);
                if (in2) r = addq(x_in2(k), r, q);
                out[u0 + E * k] = shoup(r, q2i, q2s, q);
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            u64 r = shoup(subq(x_in(k), fwd_final<SMALL>(tb[rsw<LE>(u0 + E * k, blk)], mcq), q), qi, qs, q);
            if (a.epi_acc) r = addq(r, out[u0 + E * k], q);
            out[u0 + E * k] = r;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < E; ++k) xb[u0 + E * k] = fwd_final<SMALL>(tb[rsw<LE>(u0 + E * k, blk)], mcq);
}

// ---------------------------------------------------------------------------
// Row passes for small launches at N = 2^16 (R = 256 words per row): 64
// threads per row, 4 words per thread, 4 rounds of 2 stages with an LDS
// exchange between rounds.  A thread's chain of dependent work is a quarter
// of the radix-16 pass's, which is what bounds a launch of a few limb
// polynomials.  Same stages, same twiddles, same butterflies in the same
// order as k_fwd_rows2 / k_inv_rows2, so the words are the same.
// ---------------------------------------------------------------------------
constexpr int kRowT = 64, kRowsPerBlk = kThreads / kRowT;

// word index within the row of element k (< 4) of thread t in a round whose
// two stages pair words 2^lo and 2^(lo+1) apart: bits lo, lo+1 are k
__device__ __forceinline__ int row4_idx(int t, int k, int lo) {
    return ((t >> lo) << (lo + 2)) | (k << lo) | (t & ((1 << lo) - 1));
}

template <bool SMALL, bool EPI>
__device__ __forceinline__ void k_fwd_rows4_body(const NttLaunch &a, u64 *tile) {
    constexpr int LR = 8, R = 256;
    const int s = a.map.storage(blockIdx.z);
    if (own_skip(a, s, blockIdx.y)) return;
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    const ModConst mcq = a.mods[mi];
    u64 *x = a.data + blockIdx.y * a.poly_stride + (size_t)s * a.N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * a.N;
    const int blk = threadIdx.x / kRowT, t = threadIdx.x % kRowT;
    const int gb = blockIdx.x * kRowsPerBlk + blk;
    u64 *xb = x + (size_t)gb * R;
    u64 *tb = tile + blk * R;
    u64 v[4];
    // forward (CT) stages sl = 0..7 pair words 2^(7 - sl) apart; round r
    // takes sl = 2r (k, k+2) and 2r+1 (k, k+1) on words row4_idx(t, k, 6 - 2r)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = xb[row4_idx(t, k, 6)];
    // every twiddle of the thread, fetched at once: in stage 2r both pairs
    // share one (their words differ below bit 8 - 2r), stage 2r+1 takes two
    auto twi = [&](int sl, int k, int lo) { return (1 << (LR + sl)) + (gb << sl) + (row4_idx(t, k, lo) >> (LR - sl)); };
    ulonglong2 tws[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 6 - 2 * r;
        tws[r][0] = tw[twi(2 * r, 0, lo)];
        tws[r][1] = tw[twi(2 * r + 1, 0, lo)];
        tws[r][2] = tw[twi(2 * r + 1, 2, lo)];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 6 - 2 * r;
        if (r > 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = tb[row4_idx(t, k, lo)];
        }
        ct_bfly<SMALL>(v[0], v[2], tws[r][0].x, tws[r][0].y, q, q4, nq);
        ct_bfly<SMALL>(v[1], v[3], tws[r][0].x, tws[r][0].y, q, q4, nq);
        ct_bfly<SMALL>(v[0], v[1], tws[r][1].x, tws[r][1].y, q, q4, nq);
        ct_bfly<SMALL>(v[2], v[3], tws[r][2].x, tws[r][2].y, q, q4, nq);
        if (r < 3) {  // a thread writes back the words it read this round
#pragma unroll
            for (int k = 0; k < 4; ++k) tb[row4_idx(t, k, lo)] = v[k];
            __syncthreads();
        }
    }
    // the last round's words are row4_idx(t, k, 0) = 4 t + k
    const size_t w = (size_t)s * a.N + (size_t)gb * R + 4 * t;
    if constexpr (EPI) {  // rescale / ModDown finish: (in - y) qinv (+ out)
        const u64 *in = a.epi_in + blockIdx.y * a.epi_in_stride + w;
        u64 *out = a.epi_out + blockIdx.y * a.epi_out_stride + w;
        const u64 qi = a.qinv[mi], qs = a.qinv_sh[mi];
        if (a.qinv2) {
            const u64 *in2 = a.epi_in2 ? a.epi_in2 + blockIdx.y * a.epi_in2_stride + w : nullptr;
            const u64 q2i = a.qinv2[mi], q2s = a.qinv2_sh[mi];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                u64 r = shoup(subq(in[k], fwd_final<SMALL>(v[k], mcq), q), qi, qs, q);
                if (in2) r = addq(in2[k], r, q);
                out[k] = shoup(r, q2i, q2s, q);
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            u64 r = shoup(subq(in[k], fwd_final<SMALL>(v[k], mcq), q), qi, qs, q);
            if (a.epi_acc) r = addq(r, out[k], q);
            out[k] = r;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) xb[4 * t + k] = fwd_final<SMALL>(v[k], mcq);
    }
}

template <bool EPI>
__global__ __launch_bounds__(kThreads) void k_fwd_rows4(NttLaunch a) {
    __shared__ u64 tile[kRowsPerBlk * 256];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.z))].q;
    if (qb < kSmallQ)
        k_fwd_rows4_body<true, EPI>(a, tile);
    else
        k_fwd_rows4_body<false, EPI>(a, tile);
}

template <bool SMALL>
__device__ __forceinline__ void k_inv_rows4_body(const NttLaunch &a, u64 *tile) {
    constexpr int LR = 8, R = 256;
    const int s = a.map.storage(blockIdx.z);
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    const int N = a.N;
    u64 *x = a.data + blockIdx.y * a.poly_stride + (size_t)s * N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * N;
    const int blk = threadIdx.x / kRowT, t = threadIdx.x % kRowT;
    const int gb = blockIdx.x * kRowsPerBlk + blk;
    u64 *xb = x + (size_t)gb * R;
    const u64 *xsb = (a.src ? a.src + blockIdx.y * a.src_poly_stride + (size_t)s * N : x) + (size_t)gb * R;
    u64 *tb = tile + blk * R;
    u64 v[4];
    // inverse (GS) stages lt = 0..7 pair words 2^lt apart; round r takes
    // lt = 2r (k, k+1) and 2r+1 (k, k+2) on words row4_idx(t, k, 2r)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = xsb[row4_idx(t, k, 0)];
    // every twiddle of the thread, fetched at once: stage 2r takes two (pairs
    // (0,1), (2,3)), in stage 2r+1 the pairs (0,2), (1,3) share one
    auto twi = [&](int lt, int k, int lo) {
        return (N >> (lt + 1)) + (gb << (LR - lt - 1)) + (row4_idx(t, k, lo) >> (lt + 1));
    };
    ulonglong2 tws[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 2 * r;
        tws[r][0] = tw[twi(2 * r, 0, lo)];
        tws[r][1] = tw[twi(2 * r, 2, lo)];
        tws[r][2] = tw[twi(2 * r + 1, 0, lo)];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 2 * r, lt = 2 * r;
        if (r > 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = tb[row4_idx(t, k, lo)];
        }
        gs_bfly<SMALL>(v[0], v[1], tws[r][0].x, tws[r][0].y, q, q4, nq, q << (lt + 1));
        gs_bfly<SMALL>(v[2], v[3], tws[r][1].x, tws[r][1].y, q, q4, nq, q << (lt + 1));
        gs_bfly<SMALL>(v[0], v[2], tws[r][2].x, tws[r][2].y, q, q4, nq, q << (lt + 2));
        gs_bfly<SMALL>(v[1], v[3], tws[r][2].x, tws[r][2].y, q, q4, nq, q << (lt + 2));
        if (r < 3) {
#pragma unroll
            for (int k = 0; k < 4; ++k) tb[row4_idx(t, k, lo)] = v[k];
            __syncthreads();
        }
    }
    // the last round's words are row4_idx(t, k, 6) = t + 64 k
#pragma unroll
    for (int k = 0; k < 4; ++k) xb[t + 64 * k] = v[k];
}

__global__ __launch_bounds__(kThreads) void k_inv_rows4(NttLaunch a) {
    __shared__ u64 tile[kRowsPerBlk * 256];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.z))].q;
    if (qb < kSmallQ)
        k_inv_rows4_body<true>(a, tile);
    else
        k_inv_rows4_body<false>(a, tile);
}

// Column passes for small launches at N = 2^16: the same 4-words-per-thread
// rounds down each column (64 threads per column), 16 columns per block of
// 1024 threads so that a wave's loads cover 16 consecutive columns.
constexpr int kColT = 64, kColsPerBlk = 16, kColThreads = kColT * kColsPerBlk;

template <bool SMALL>
__device__ __forceinline__ void k_fwd_cols4_body(const NttLaunch &a, u64 *tile) {
    constexpr int LR = 8, R = 256;
    const int s = a.map.storage(blockIdx.y);
    if (own_skip(a, s, blockIdx.z)) return;
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * a.N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * a.N;
    const int c = threadIdx.x % kColsPerBlk, g = threadIdx.x / kColsPerBlk;
    const int col = blockIdx.x * kColsPerBlk + c;
    const u64 *xs = a.src ? a.src + blockIdx.z * a.src_poly_stride + (a.pre_top >= 0 ? 0 : (size_t)s * a.N) : x;
    u64 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = xs[col + (size_t)row4_idx(g, k, 6) * R];
    if (a.pre_top >= 0) {  // centered residue of the top limb in this limb
        const u64 qt = a.mods[a.pre_top].q;
        const ModConst mc = a.mods[mi];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (v[k] > (qt >> 1)) {
                const u64 neg = reduce64(qt - v[k], mc);
                v[k] = neg ? mc.q - neg : 0;
            } else {
                v[k] = reduce64(v[k], mc);
            }
        }
    }
    // stages st = 0..7 pair rows 2^(7 - st) apart, twiddle (1 << st) + (j >> (8 - st))
    ulonglong2 tws[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 6 - 2 * r;
        tws[r][0] = tw[(1 << (2 * r)) + (row4_idx(g, 0, lo) >> (LR - 2 * r))];
        tws[r][1] = tw[(1 << (2 * r + 1)) + (row4_idx(g, 0, lo) >> (LR - 2 * r - 1))];
        tws[r][2] = tw[(1 << (2 * r + 1)) + (row4_idx(g, 2, lo) >> (LR - 2 * r - 1))];
    }
    __builtin_amdgcn_sched_barrier(0);
    u64 *tc = tile + c;  // column c of the tile, rows kColsPerBlk words apart
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 6 - 2 * r;
        if (r > 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = tc[row4_idx(g, k, lo) * kColsPerBlk];
        }
        ct_bfly<SMALL>(v[0], v[2], tws[r][0].x, tws[r][0].y, q, q4, nq);
        ct_bfly<SMALL>(v[1], v[3], tws[r][0].x, tws[r][0].y, q, q4, nq);
        ct_bfly<SMALL>(v[0], v[1], tws[r][1].x, tws[r][1].y, q, q4, nq);
        ct_bfly<SMALL>(v[2], v[3], tws[r][2].x, tws[r][2].y, q, q4, nq);
        if (r < 3) {  // a thread writes back the words it read this round
#pragma unroll
            for (int k = 0; k < 4; ++k) tc[row4_idx(g, k, lo) * kColsPerBlk] = v[k];
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[col + (size_t)(4 * g + k) * R] = v[k];
}

__global__ __launch_bounds__(kColThreads) void k_fwd_cols4(NttLaunch a) {
    __shared__ u64 tile[256 * kColsPerBlk];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.y))].q;
    if (qb < kSmallQ)
        k_fwd_cols4_body<true>(a, tile);
    else
        k_fwd_cols4_body<false>(a, tile);
}

template <bool SMALL>
__device__ __forceinline__ void k_inv_cols4_body(const NttLaunch &a, u64 *tile) {
    constexpr int LR = 8, R = 256;
    const int s = a.map.storage(blockIdx.y);
    const int mi = a.map.modidx(s);
    const ModConst mc = a.mods[mi];
    const u64 q = mc.q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    const int N = a.N;
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * N;
    const int c = threadIdx.x % kColsPerBlk, g = threadIdx.x / kColsPerBlk;
    const int col = blockIdx.x * kColsPerBlk + c;
    u64 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = x[col + (size_t)(4 * g + k) * R];
    // stages ltp = 0..7 pair rows 2^ltp apart, twiddle (N >> (9 + ltp)) + (j >> (ltp + 1))
    ulonglong2 tws[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 2 * r;
        tws[r][0] = tw[(N >> (LR + 2 * r + 1)) + (row4_idx(g, 0, lo) >> (2 * r + 1))];
        tws[r][1] = tw[(N >> (LR + 2 * r + 1)) + (row4_idx(g, 2, lo) >> (2 * r + 1))];
        tws[r][2] = tw[(N >> (LR + 2 * r + 2)) + (row4_idx(g, 0, lo) >> (2 * r + 2))];
    }
    __builtin_amdgcn_sched_barrier(0);
    u64 *tc = tile + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = 2 * r, lt = LR + 2 * r;
        if (r > 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = tc[row4_idx(g, k, lo) * kColsPerBlk];
        }
        gs_bfly<SMALL>(v[0], v[1], tws[r][0].x, tws[r][0].y, q, q4, nq, q << (lt + 1));
        gs_bfly<SMALL>(v[2], v[3], tws[r][1].x, tws[r][1].y, q, q4, nq, q << (lt + 1));
        gs_bfly<SMALL>(v[0], v[2], tws[r][2].x, tws[r][2].y, q, q4, nq, q << (lt + 2));
        gs_bfly<SMALL>(v[1], v[3], tws[r][2].x, tws[r][2].y, q, q4, nq, q << (lt + 2));
        if (r < 3) {
#pragma unroll
            for (int k = 0; k < 4; ++k) tc[row4_idx(g, k, lo) * kColsPerBlk] = v[k];
            __syncthreads();
        }
    }
    // the last round's rows are row4_idx(g, k, 6) = g + 64 k
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u64 r = shoup_lazy(v[k], mc.ninv, mc.ninv_sh, q);
        x[col + (size_t)(g + 64 * k) * R] = r >= q ? r - q : r;
    }
}

__global__ __launch_bounds__(kColThreads) void k_inv_cols4(NttLaunch a) {
    __shared__ u64 tile[256 * kColsPerBlk];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.y))].q;
    if (qb < kSmallQ)
        k_inv_cols4_body<true>(a, tile);
    else
        k_inv_cols4_body<false>(a, tile);
}

// EPI: the launch carries an epilogue (epi_out set)
template <int LE, bool EPI>
__global__ __launch_bounds__(kThreads) void k_fwd_rows2(NttLaunch a) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, BLKS = kThreads / E;
    __shared__ u64 tile[BLKS * R];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.z))].q;
    if (qb < kSmallQ)
        k_fwd_rows2_body<LE, true, EPI>(a, tile);
    else
        k_fwd_rows2_body<LE, false, EPI>(a, tile);
}

template <int LE, bool SMALL>
__device__ __forceinline__ void k_inv_rows2_body(const NttLaunch &a, u64 *tile) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, BLKS = kThreads / E;
    const int s = a.map.storage(blockIdx.z);
    const int mi = a.map.modidx(s);
    const u64 q = a.mods[mi].q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    const int N = a.N;
    u64 *x = a.data + blockIdx.y * a.poly_stride + (size_t)s * N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * N;
    const int blk = threadIdx.x / E, u0 = threadIdx.x % E;
    const int gb = blockIdx.x * BLKS + blk;
    u64 *xb = x + (size_t)gb * R;
    const u64 *xsb = (a.src ? a.src + blockIdx.y * a.src_poly_stride + (size_t)s * N : x) + (size_t)gb * R;
    u64 *tb = tile + blk * R;
    u64 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) tb[rsw<LE>(u0 + E * k, blk)] = xsb[u0 + E * k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = tb[rsw<LE>(E * u0 + k, blk)];
#pragma unroll
    for (int lt = 0; lt < LE; ++lt) {
        const int half = 1 << lt;
        NTT_STAGE_TW(false, (N >> (lt + 1)) + (gb << (LR - lt - 1)) + (u0 << (LE - lt - 1)), lt + 1)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(false, k, lt + 1);
                gs_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq, q << (lt + 1));
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) tb[rsw<LE>(E * u0 + k, blk)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = tb[rsw<LE>(u0 + E * k, blk)];
#pragma unroll
    for (int lt = LE; lt < LR; ++lt) {
        const int half = 1 << (lt - LE);
        NTT_STAGE_TW(false, (N >> (lt + 1)) + (gb << (LR - lt - 1)), lt + 1 - LE)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(false, k, lt + 1 - LE);
                gs_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq, q << (lt + 1));
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) xb[u0 + E * k] = v[k];
}

template <int LE>
__global__ __launch_bounds__(kThreads) void k_inv_rows2(NttLaunch a) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, BLKS = kThreads / E;
    __shared__ u64 tile[BLKS * R];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.z))].q;
    if (qb < kSmallQ)
        k_inv_rows2_body<LE, true>(a, tile);
    else
        k_inv_rows2_body<LE, false>(a, tile);
}

template <int LE, bool SMALL>
__device__ __forceinline__ void k_inv_cols2_body(const NttLaunch &a, u64 *tile) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, COLS = kThreads / E;
    const int s = a.map.storage(blockIdx.y);
    const int mi = a.map.modidx(s);
    const ModConst mc = a.mods[mi];
    const u64 q = mc.q, q4 = 4 * q;
    const u64 nq = opaque_neg(q);
    const int N = a.N;
    u64 *x = a.data + blockIdx.z * a.poly_stride + (size_t)s * N;
    const ulonglong2 *tw = a.tw2 + (size_t)mi * N;
    const int c = threadIdx.x % COLS, g = threadIdx.x / COLS;
    const int col = blockIdx.x * COLS + c;
    u64 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = x[col + (size_t)(E * g + k) * R];
#pragma unroll
    for (int ltp = 0; ltp < LE; ++ltp) {
        const int half = 1 << ltp;
        NTT_STAGE_TW(false, (N >> (LR + ltp + 1)) + (g << (LE - ltp - 1)), ltp + 1)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(false, k, ltp + 1);
                gs_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq, q << (LR + ltp + 1));
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) tile[csw<LE>(E * g + k) * COLS + c] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = tile[csw<LE>(g + E * k) * COLS + c];
#pragma unroll
    for (int ltp = LE; ltp < LR; ++ltp) {
        const int half = 1 << (ltp - LE);
        NTT_STAGE_TW(false, N >> (LR + ltp + 1), ltp + 1 - LE)
#pragma unroll
        for (int k = 0; k < E; ++k)
            if ((k & half) == 0) {
                const ulonglong2 t2 = NTT_TW(false, k, ltp + 1 - LE);
                gs_bfly<SMALL>(v[k], v[k + half], t2.x, t2.y, q, q4, nq, q << (LR + ltp + 1));
            }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
        u64 r = shoup_lazy(v[k], mc.ninv, mc.ninv_sh, q);
        x[col + (size_t)(g + E * k) * R] = r >= q ? r - q : r;
    }
}

template <int LE>
__global__ __launch_bounds__(kThreads) void k_inv_cols2(NttLaunch a) {
    constexpr int E = 1 << LE, LR = 2 * LE, R = 1 << LR, COLS = kThreads / E;
    __shared__ u64 tile[R * COLS];
    const u64 qb = a.mods[a.map.modidx(a.map.storage(blockIdx.y))].q;
    if (qb < kSmallQ)
        k_inv_cols2_body<LE, true>(a, tile);
    else
        k_inv_cols2_body<LE, false>(a, tile);
}

LimbMap qmap_all() { return LimbMap{0, INT_MAX, 0, INT_MAX, 0}; }

NttLaunch make_launch(const fr_ctx *c, u64 *data, const LimbMap &map, size_t poly_stride, bool inverse,
                      const u64 *src, size_t src_poly_stride) {
    NttLaunch a;
    a.data = data;
    a.poly_stride = poly_stride;
    a.src = src;
    a.src_poly_stride = src_poly_stride;
    a.N = c->N;
    a.logN = c->logN;
    a.s1 = c->logN / 2;
    a.map = map;
    a.tw = inverse ? c->d_itw : c->d_tw;
    a.tw_sh = inverse ? c->d_itw_sh : c->d_tw_sh;
    a.tw2 = reinterpret_cast<const ulonglong2 *>(inverse ? c->d_itw2 : c->d_tw2);
    a.mods = c->d_mod;
    a.pre_top = -1;
    a.epi_acc = 0;
    a.epi_in2 = nullptr;
    a.epi_in2_stride = 0;
    a.qinv2 = a.qinv2_sh = nullptr;
    a.epi_out = nullptr;
    a.epi_in = nullptr;
    a.epi_out_stride = a.epi_in_stride = 0;
    a.qinv = a.qinv_sh = nullptr;
    a.own_alpha = 0;
    a.own_ndig = 1;
    a.own_nlq = 0;
    return a;
}

// limb polynomials up to which the N = 2^16 passes take 4 words per thread
// (a launch this small is bound by one thread's chain of work): the
// context's tuning knobs, set from measured pass durations
void fwd_cols16(const fr_ctx *c, const NttLaunch &a, int npoly, int nlimbs, dim3 g) {
    if (npoly * nlimbs <= c->tune[FR_TUNE_NTT_FWD_COLS4])
        hipLaunchKernelGGL(k_fwd_cols4, g, dim3(kColThreads), 0, c->stream, a);
    else
        hipLaunchKernelGGL(k_fwd_cols2<4>, g, dim3(kThreads), 0, c->stream, a);
}

void inv_cols16(const fr_ctx *c, const NttLaunch &a, int npoly, int nlimbs, dim3 g) {
    if (npoly * nlimbs <= c->tune[FR_TUNE_NTT_INV_COLS4])
        hipLaunchKernelGGL(k_inv_cols4, g, dim3(kColThreads), 0, c->stream, a);
    else
        hipLaunchKernelGGL(k_inv_cols2<4>, g, dim3(kThreads), 0, c->stream, a);
}

template <bool EPI>
void fwd_rows16(const fr_ctx *c, const NttLaunch &a, int npoly, int nlimbs, dim3 gr) {
    if (npoly * nlimbs <= c->tune[FR_TUNE_NTT_FWD_ROWS4])
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_rows4<EPI>), dim3(256 / kRowsPerBlk, npoly, nlimbs), dim3(kThreads),
                           0, c->stream, a);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_rows2<4, EPI>), gr, dim3(kThreads), 0, c->stream, a);
}

void inv_rows16(const fr_ctx *c, const NttLaunch &a, int npoly, int nlimbs, dim3 gr) {
    if (npoly * nlimbs <= c->tune[FR_TUNE_NTT_INV_ROWS4])
        hipLaunchKernelGGL(k_inv_rows4, dim3(256 / kRowsPerBlk, npoly, nlimbs), dim3(kThreads), 0, c->stream, a);
    else
        hipLaunchKernelGGL(k_inv_rows2<4>, gr, dim3(kThreads), 0, c->stream, a);
}

}  // namespace

namespace frk {

bool ntt_own_skip_ok(const fr_ctx *c) { return c->logN == 16 || c->logN == 12; }

void ntt_fwd(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly, size_t poly_stride,
             const u64 *src, size_t src_poly_stride, int own_alpha, int own_ndig, int own_nlq) {
    if (nlimbs <= 0 || npoly <= 0) return;
    const bool own = own_alpha > 0 && ntt_own_skip_ok(c);
    // limb polynomials transformed (a digit's own limbs are not)
    const double lp = (double)nlimbs * npoly - (own ? (double)(npoly / own_ndig) * own_nlq : 0.0);
    ProfScope ps(c, K_NTT, 16.0 * lp * c->N);
    NttLaunch a = make_launch(c, data, map, poly_stride, false, src, src_poly_stride);
    if (own) {
        a.own_alpha = own_alpha;
        a.own_ndig = own_ndig;
        a.own_nlq = own_nlq;
    }
    if (c->logN == 16 || c->logN == 12) {
        const int LE = c->logN / 4, E = 1 << LE, R = 1 << (2 * LE);
        // the row passes walk every polynomial of one limb before the next
        // limb, so the limb's large-stage twiddles stay in L2
        dim3 g(R / (kThreads / E), nlimbs, npoly), gr(R / (kThreads / E), npoly, nlimbs);
        if (LE == 4) {
            fwd_cols16(c, a, npoly, nlimbs, g);
            fwd_rows16<false>(c, a, npoly, nlimbs, gr);
        } else {
            hipLaunchKernelGGL(k_fwd_cols2<3>, g, dim3(kThreads), 0, c->stream, a);
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_rows2<3, false>), gr, dim3(kThreads), 0, c->stream, a);
        }
        return;
    }
    const int lr = a.s1, lc = a.logN - a.s1;
    const int lcols = std::min(12 - lr, lc), lblks = std::min(12 - lc, lr);
    dim3 g1(1 << (lc - lcols), nlimbs, npoly), g2(1 << (lr - lblks), nlimbs, npoly);
    hipLaunchKernelGGL(k_fwd_cols, g1, dim3(kThreads), 0, c->stream, a);
    hipLaunchKernelGGL(k_fwd_rows, g2, dim3(kThreads), 0, c->stream, a);
}

bool ntt_fwd_rescale(const fr_ctx *c, u64 *tmp, int l, int npoly, const u64 *xtop, const u64 *in, size_t in_stride,
                     u64 *out, size_t out_stride) {
    if (c->logN != 16 && c->logN != 12) return false;
    if (l <= 0 || npoly <= 0) return true;
    ProfScope ps(c, K_NTT, 16.0 * l * npoly * c->N);
    NttLaunch a = make_launch(c, tmp, qmap_all(), (size_t)l * c->N, false, xtop, (size_t)c->N);
    a.pre_top = l;
    a.epi_out = out;
    a.epi_in = in;
    a.epi_out_stride = out_stride;
    a.epi_in_stride = in_stride;
    a.qinv = c->d_rescale + (size_t)l * (c->L + 1) * 2;
    a.qinv_sh = a.qinv + (c->L + 1);
    const int LE = c->logN / 4, E = 1 << LE, R = 1 << (2 * LE);
    dim3 g(R / (kThreads / E), l, npoly), gr(R / (kThreads / E), npoly, l);
    if (LE == 4) {
        fwd_cols16(c, a, npoly, (int)gr.z, g);
        fwd_rows16<true>(c, a, npoly, (int)gr.z, gr);
    } else {
        hipLaunchKernelGGL(k_fwd_cols2<3>, g, dim3(kThreads), 0, c->stream, a);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_rows2<3, true>), gr, dim3(kThreads), 0, c->stream, a);
    }
    return true;
}

bool ntt_fwd_moddown(const fr_ctx *c, u64 *V, int level, int npoly, const u64 *U, size_t su, u64 *out, size_t so,
                     bool accumulate) {
    if (c->logN != 16 && c->logN != 12) return false;
    const int nl = level + 1;
    ProfScope ps(c, K_NTT, 16.0 * nl * npoly * c->N);
    NttLaunch a = make_launch(c, V, qmap_all(), (size_t)nl * c->N, false, nullptr, 0);
    a.epi_out = out;
    a.epi_in = U;
    a.epi_out_stride = so;
    a.epi_in_stride = su;
    a.epi_acc = accumulate;
    a.qinv = c->d_moddown + 2 * c->nP + (size_t)(c->L + 1) * c->nP;  // P^-1 mod q_i, then its companions
    a.qinv_sh = a.qinv + (c->L + 1);
    const int LE = c->logN / 4, E = 1 << LE, R = 1 << (2 * LE);
    dim3 g(R / (kThreads / E), nl, npoly), gr(R / (kThreads / E), npoly, nl);
    if (LE == 4) {
        fwd_cols16(c, a, npoly, (int)gr.z, g);
        fwd_rows16<true>(c, a, npoly, (int)gr.z, gr);
    } else {
        hipLaunchKernelGGL(k_fwd_cols2<3>, g, dim3(kThreads), 0, c->stream, a);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_rows2<3, true>), gr, dim3(kThreads), 0, c->stream, a);
    }
    return true;
}

bool ntt_fwd_relin_rescale(const fr_ctx *c, u64 *Z, int l, int npoly, const u64 *U, size_t su, const u64 *d,
                           size_t sd, u64 *out, size_t so) {
    if (c->logN != 16 && c->logN != 12) return false;
    ProfScope ps(c, K_NTT, 16.0 * l * npoly * c->N);
    NttLaunch a = make_launch(c, Z, qmap_all(), (size_t)l * c->N, false, nullptr, 0);
    a.epi_out = out;
    a.epi_in = U;
    a.epi_out_stride = so;
    a.epi_in_stride = su;
    a.epi_in2 = d;
    a.epi_in2_stride = sd;
    const size_t rtab = (size_t)(c->L + 1) * (c->L + 1) * 2;
    if (d) {
        a.qinv = c->d_moddown + 2 * c->nP + (size_t)(c->L + 1) * c->nP;  // P^-1 mod q_i and companions
        a.qinv_sh = a.qinv + (c->L + 1);
        a.qinv2 = c->d_rescale + (size_t)l * (c->L + 1) * 2;  // q_l^-1 mod q_i and companions
        a.qinv2_sh = a.qinv2 + (c->L + 1);
    } else {
        // no d term: one product by (P q_l)^-1 mod q_i (the same canonical words)
        a.qinv = c->d_rescale + rtab + (size_t)l * (c->L + 1) * 2;
        a.qinv_sh = a.qinv + (c->L + 1);
    }
    const int LE = c->logN / 4, E = 1 << LE, R = 1 << (2 * LE);
    dim3 g(R / (kThreads / E), l, npoly), gr(R / (kThreads / E), npoly, l);
    if (LE == 4) {
        fwd_cols16(c, a, npoly, (int)gr.z, g);
        fwd_rows16<true>(c, a, npoly, (int)gr.z, gr);
    } else {
        hipLaunchKernelGGL(k_fwd_cols2<3>, g, dim3(kThreads), 0, c->stream, a);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_rows2<3, true>), gr, dim3(kThreads), 0, c->stream, a);
    }
    return true;
}

void ntt_inv(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly, size_t poly_stride,
             const u64 *src, size_t src_poly_stride) {
    if (nlimbs <= 0 || npoly <= 0) return;
    ProfScope ps(c, K_NTT, 16.0 * nlimbs * npoly * c->N);
    NttLaunch a = make_launch(c, data, map, poly_stride, true, src, src_poly_stride);
    if (c->logN == 16 || c->logN == 12) {
        const int LE = c->logN / 4, E = 1 << LE, R = 1 << (2 * LE);
        dim3 g(R / (kThreads / E), nlimbs, npoly), gr(R / (kThreads / E), npoly, nlimbs);
        if (LE == 4) {
            inv_rows16(c, a, npoly, nlimbs, gr);
            inv_cols16(c, a, npoly, nlimbs, g);
        } else {
            hipLaunchKernelGGL(k_inv_rows2<3>, gr, dim3(kThreads), 0, c->stream, a);
            hipLaunchKernelGGL(k_inv_cols2<3>, g, dim3(kThreads), 0, c->stream, a);
        }
        return;
    }
    const int lr = a.s1, lc = a.logN - a.s1;
    const int lcols = std::min(12 - lr, lc), lblks = std::min(12 - lc, lr);
    dim3 g1(1 << (lc - lcols), nlimbs, npoly), g2(1 << (lr - lblks), nlimbs, npoly);
    hipLaunchKernelGGL(k_inv_rows, g2, dim3(kThreads), 0, c->stream, a);
    hipLaunchKernelGGL(k_inv_cols, g1, dim3(kThreads), 0, c->stream, a);
}

}  // namespace frk
