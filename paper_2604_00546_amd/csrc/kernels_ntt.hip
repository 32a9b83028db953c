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
    int N, logN, s1;
    LimbMap map;
    const u64 *tw, *tw_sh;
    const ModConst *mods;
};

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
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        int r = idx >> lcols, c = idx & (COLS - 1);
        tile[idx] = x[c0 + c + ((size_t)r << lc)];
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
    for (int idx = threadIdx.x; idx < total; idx += kThreads) tile[idx] = x[idx];
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

NttLaunch make_launch(const fr_ctx *c, u64 *data, const LimbMap &map, size_t poly_stride, bool inverse) {
    NttLaunch a;
    a.data = data;
    a.poly_stride = poly_stride;
    a.N = c->N;
    a.logN = c->logN;
    a.s1 = c->logN / 2;
    a.map = map;
    a.tw = inverse ? c->d_itw : c->d_tw;
    a.tw_sh = inverse ? c->d_itw_sh : c->d_tw_sh;
    a.mods = c->d_mod;
    return a;
}

}  // namespace

namespace frk {

void ntt_fwd(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly, size_t poly_stride) {
    if (nlimbs <= 0 || npoly <= 0) return;
    ProfScope ps(c, K_NTT, 16.0 * nlimbs * npoly * c->N);
    NttLaunch a = make_launch(c, data, map, poly_stride, false);
    const int lr = a.s1, lc = a.logN - a.s1;
    const int lcols = std::min(12 - lr, lc), lblks = std::min(12 - lc, lr);
    dim3 g1(1 << (lc - lcols), nlimbs, npoly), g2(1 << (lr - lblks), nlimbs, npoly);
    hipLaunchKernelGGL(k_fwd_cols, g1, dim3(kThreads), 0, c->stream, a);
    hipLaunchKernelGGL(k_fwd_rows, g2, dim3(kThreads), 0, c->stream, a);
}

void ntt_inv(const fr_ctx *c, u64 *data, int nlimbs, const LimbMap &map, int npoly, size_t poly_stride) {
    if (nlimbs <= 0 || npoly <= 0) return;
    ProfScope ps(c, K_NTT, 16.0 * nlimbs * npoly * c->N);
    NttLaunch a = make_launch(c, data, map, poly_stride, true);
    const int lr = a.s1, lc = a.logN - a.s1;
    const int lcols = std::min(12 - lr, lc), lblks = std::min(12 - lc, lr);
    dim3 g1(1 << (lc - lcols), nlimbs, npoly), g2(1 << (lr - lblks), nlimbs, npoly);
    hipLaunchKernelGGL(k_inv_rows, g2, dim3(kThreads), 0, c->stream, a);
    hipLaunchKernelGGL(k_inv_cols, g1, dim3(kThreads), 0, c->stream, a);
}

}  // namespace frk
