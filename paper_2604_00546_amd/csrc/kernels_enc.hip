// kernels_enc.hip -- encoding (§3.2), randomness and database layout kernels.
//
// Encoding is the inverse canonical embedding done with an FP64 complex FFT
// of length N: slot j lives at the root zeta^(5^j mod 2N) = zeta^(2 t_j + 1)
// and its conjugate at zeta^(2 (N - 1 - t_j) + 1); with w[t] the value at
// zeta^(2t+1), m_k = Re(zeta^-k * DFT(w)[k]) / N.  Decoding evaluates the
// lifted coefficients back: slot j = sum_k (m_k zeta^k) exp(2 pi i t_j k / N).
// FP64 is used only here; everything after rounding is exact integer work.
#include <algorithm>

#include "fr_core.h"

namespace {

constexpr int kT = 256;

struct Cdt {
    u64 v[20];
};

// ---- Philox-4x64-10 (Salmon et al., SC'11) ----
__device__ __forceinline__ void philox(u64 c[4], u64 k0, u64 k1) {
    const u64 M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const u64 W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const u64 lo0 = M0 * c[0], hi0 = mulhi64(M0, c[0]);
        const u64 lo1 = M1 * c[2], hi1 = mulhi64(M1, c[2]);
        const u64 n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// uniform residues: block b of limb with global index gm gives coefficients
// 2b, 2b+1 as the 128-bit words (r1:r0), (r3:r2) reduced mod q
__global__ __launch_bounds__(kT) void k_sample_uniform(u64 *out, u64 seed, u64 poly, LimbMap map, int N,
                                                       const ModConst *mods) {
    const int b = blockIdx.x * kT + threadIdx.x;
    if (b >= N / 2) return;
    const int s = map.storage(blockIdx.y);
    const int gm = map.modidx(s);
    const ModConst m = mods[gm];
    u64 c[4] = {(u64)b, (u64)gm, poly, 0};
    philox(c, seed, 1);
    u64 *o = out + (size_t)s * N + 2 * b;
    o[0] = reduce128(c[0], c[1], m);
    o[1] = reduce128(c[2], c[3], m);
}

// small signed polynomials: kind 2 = ternary (word mod 3) - 1,
// kind 3 = Gaussian (top bit sign, low 63 bits through the CDT)
__global__ __launch_bounds__(kT) void k_sample_small(u64 *out, u64 seed, u64 poly, int kind, Cdt cdt, LimbMap map,
                                                     int nlimbs, int N, const ModConst *mods) {
    const int b = blockIdx.x * kT + threadIdx.x;
    if (b >= N / 4) return;
    u64 c[4] = {(u64)b, 0, poly, 0};
    philox(c, seed, (u64)kind);
    long long v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (kind == 2) {
            v[u] = (long long)(c[u] % 3ull) - 1;
        } else {
            const u64 sign = c[u] >> 63, x = c[u] & 0x7FFFFFFFFFFFFFFFull;
            int t = 0;
            while (t < 19 && x >= cdt.v[t]) ++t;
            v[u] = (sign && t) ? -(long long)t : (long long)t;
        }
    }
    for (int y = 0; y < nlimbs; ++y) {
        const int s = map.storage(y);
        const u64 q = mods[map.modidx(s)].q;
        u64 *o = out + (size_t)s * N + 4 * b;
#pragma unroll
        for (int u = 0; u < 4; ++u) o[u] = v[u] >= 0 ? (u64)v[u] : q - (u64)(-v[u]);
    }
}

// ---- FP64 FFT (radix-2 decimation in time; input in bit-reversed order) ----
__global__ __launch_bounds__(kT) void k_fft_stage(double2 *w, int N, int lhalf, int batch, const double *tw,
                                                  int inverse) {
    const int idx = blockIdx.x * kT + threadIdx.x;
    const int half_total = N / 2;
    if (idx >= half_total * batch) return;
    const int vb = idx / half_total, bf = idx % half_total;
    const int half = 1 << lhalf;
    const int grp = bf >> lhalf, j = bf & (half - 1);
    double2 *x = w + (size_t)vb * N + ((size_t)grp << (lhalf + 1));
    const int ti = j * (N >> (lhalf + 1));
    const double cr = tw[2 * ti], ci = inverse ? -tw[2 * ti + 1] : tw[2 * ti + 1];
    const double2 a = x[j], b = x[j + half];
    const double2 bt = make_double2(b.x * cr - b.y * ci, b.x * ci + b.y * cr);
    x[j] = make_double2(a.x + bt.x, a.y + bt.y);
    x[j + half] = make_double2(a.x - bt.x, a.y - bt.y);
}

__global__ __launch_bounds__(kT) void k_enc_scatter(double2 *w, const double *z, int n, size_t zs, int N, int logN,
                                                    const u32 *slot_pos) {
    const int j = blockIdx.x * kT + threadIdx.x, vb = blockIdx.y;
    if (j >= N / 2) return;
    const double v = j < n ? z[vb * zs + j] : 0.0;
    const u32 t = slot_pos[j];
    double2 *x = w + (size_t)vb * N;
    x[brv(t, logN)] = make_double2(v, 0.0);
    x[brv((u32)N - 1 - t, logN)] = make_double2(v, 0.0);
}

__global__ __launch_bounds__(kT) void k_enc_round(u64 *out, const double2 *w, int N, int level, double scale,
                                                  size_t os, const double *zeta, const ModConst *mods, int *flag) {
    const int k = blockIdx.x * kT + threadIdx.x, vb = blockIdx.y;
    const double2 W = w[(size_t)vb * N + k];
    const double re = W.x * zeta[2 * k] + W.y * zeta[2 * k + 1];  // Re(conj(zeta^k) W)
    const double x = rint(re * scale / (double)N);
    long long v = 0;
    if (!(fabs(x) < 4.611686018427388e18)) {
        atomicOr(flag, 1);
    } else {
        v = (long long)x;
    }
    u64 *o = out + vb * os + k;
    for (int i = 0; i <= level; ++i) {
        const ModConst m = mods[i];
        u64 r;
        if (v >= 0) {
            r = reduce64((u64)v, m);
        } else {
            const u64 a = reduce64((u64)(-v), m);
            r = a ? m.q - a : 0;
        }
        o[(size_t)i * N] = r;
    }
}

// centered CRT lift of coefficient form m[level+1][N] to double, twisted by
// zeta^k and scattered into bit-reversed order for the decoding FFT.
// tab (per level): qhat_inv[L+1], qhat_inv_sh[L+1], qhat_mod64[L+1], inv_q[L+1], Q_mod64
__global__ __launch_bounds__(kT) void k_crt_lift(double2 *w, const u64 *m, int N, int logN, int level, int L1,
                                                 const u64 *tab, const double *zeta, const ModConst *mods, int *flag) {
    const int k = blockIdx.x * kT + threadIdx.x;
    const u64 *qhi = tab, *qhi_sh = tab + L1, *qh64 = tab + 2 * L1;
    const double *invq = reinterpret_cast<const double *>(tab + 3 * L1);
    const u64 Q64 = tab[4 * L1];
    double s = 0.0;
    u64 acc = 0;
    for (int i = 0; i <= level; ++i) {
        const u64 y = shoup(m[(size_t)i * N + k], qhi[i], qhi_sh[i], mods[i].q);
        s += (double)y * invq[i];
        acc += y * qh64[i];
    }
    const double v = rint(s);
    if (fabs(s - v) > 0.25) atomicOr(flag, 2);
    const long long x = (long long)(acc - (u64)v * Q64);
    if (x > (1ll << 62) || x < -(1ll << 62)) atomicOr(flag, 2);
    const double xd = (double)x;
    w[brv((u32)k, logN)] = make_double2(xd * zeta[2 * k], xd * zeta[2 * k + 1]);
}

__global__ __launch_bounds__(kT) void k_dec_gather(double *z, const double2 *w, int n, double scale,
                                                   const u32 *slot_pos) {
    const int j = blockIdx.x * kT + threadIdx.x;
    if (j >= n) return;
    z[j] = w[slot_pos[j]].x / scale;
}

// pre-rotated diagonal slot vectors of group g, diagonals d0 .. d0+nd-1
__global__ __launch_bounds__(kT) void k_db_slots(double *out, const float *T, int K, int ell, int B, int n1, int g,
                                                 int d0, int h) {
    const int s = blockIdx.x * kT + threadIdx.x, dd = blockIdx.y;
    if (s >= h) return;
    const int d = d0 + dd;
    const int j = d / n1;
    int src = (s - j * n1) % h;
    if (src < 0) src += h;
    double v = 0.0;
    if (src < B * ell) {
        const int b = src / ell, r = src % ell;
        const long long row = ((long long)g * B + b) * ell + r;
        if (row < K) v = (double)T[row * ell + (r + d) % ell];
    }
    out[(size_t)dd * h + s] = v;
}

void fft(const fr_ctx *c, double2 *w, int batch, bool inverse) {
    const int total = c->N / 2 * batch;
    for (int lh = 0; lh < c->logN; ++lh)
        hipLaunchKernelGGL(k_fft_stage, dim3((total + kT - 1) / kT), dim3(kT), 0, c->stream, w, c->N, lh, batch,
                           c->d_fft_w, (int)inverse);
}

}  // namespace

namespace frk {

void sample_uniform(const fr_ctx *c, u64 *out, u64 seed, u64 poly, const LimbMap &map, int nlimbs) {
    dim3 g((c->N / 2 + kT - 1) / kT, nlimbs, 1);
    hipLaunchKernelGGL(k_sample_uniform, g, dim3(kT), 0, c->stream, out, seed, poly, map, c->N, c->d_mod);
}

void sample_small(const fr_ctx *c, u64 *out, u64 seed, u64 poly, int kind, const LimbMap &map, int nlimbs) {
    Cdt cdt;
    for (int i = 0; i < 20; ++i) cdt.v[i] = c->cdt[i];
    dim3 g((c->N / 4 + kT - 1) / kT, 1, 1);
    hipLaunchKernelGGL(k_sample_small, g, dim3(kT), 0, c->stream, out, seed, poly, kind, cdt, map, nlimbs, c->N,
                       c->d_mod);
}

// z: device [batch][zstride] doubles (n used); out: batch plaintexts, ostride
// words apart, coefficient form; work: batch * N double2
void encode_slots(const fr_ctx *c, u64 *out, const double *z, int n, int level, double scale, int batch,
                  size_t zstride, size_t ostride, double *work) {
    double2 *w = reinterpret_cast<double2 *>(work);
    hipLaunchKernelGGL(k_enc_scatter, dim3((c->N / 2 + kT - 1) / kT, batch), dim3(kT), 0, c->stream, w, z, n,
                       zstride, c->N, c->logN, c->d_slot_pos);
    fft(c, w, batch, false);
    hipLaunchKernelGGL(k_enc_round, dim3(c->N / kT, batch), dim3(kT), 0, c->stream, out, w, c->N, level, scale,
                       ostride, c->d_zeta, c->d_mod, c->d_flag);
}

void decode_slots(const fr_ctx *c, double *z, const u64 *m_coeff, int level, double scale, double *work) {
    double2 *w = reinterpret_cast<double2 *>(work);
    const u64 *tab = c->d_crt + (size_t)level * (4 * (c->L + 1) + 1);
    hipLaunchKernelGGL(k_crt_lift, dim3(c->N / kT), dim3(kT), 0, c->stream, w, m_coeff, c->N, c->logN, level,
                       c->L + 1, tab, c->d_zeta, c->d_mod, c->d_flag);
    fft(c, w, 1, true);
    hipLaunchKernelGGL(k_dec_gather, dim3((c->N / 2 + kT - 1) / kT), dim3(kT), 0, c->stream, z, w, c->N / 2, scale,
                       c->d_slot_pos);
}

void db_slots(const fr_ctx *c, double *out, const float *T, int K, int ell, int B, int n1, int g, int d0, int nd) {
    const int h = c->N / 2;
    hipLaunchKernelGGL(k_db_slots, dim3((h + kT - 1) / kT, nd), dim3(kT), 0, c->stream, out, T, K, ell, B, n1, g, d0,
                       h);
}

}  // namespace frk
