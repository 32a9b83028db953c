// params.cpp -- host-side parameter math: modulus chain, roots of unity,
// per-modulus reduction constants, Galois elements, Gaussian table.
#include <cmath>
#include <cstring>

#include "fr_core.h"

namespace frh {

u64 mulmod_h(u64 a, u64 b, u64 q) { return (u64)((unsigned __int128)a * b % q); }

u64 powmod_h(u64 b, u64 e, u64 q) {
    u64 r = 1 % q;
    b %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod_h(r, b, q);
        b = mulmod_h(b, b, q);
    }
    return r;
}

u64 invmod_h(u64 a, u64 q) { return powmod_h(a % q, q - 2, q); }

u64 shoup_companion(u64 w, u64 q) { return (u64)(((unsigned __int128)w << 64) / q); }

// Miller-Rabin with the prime bases up to 37: deterministic below 3.3e24.
bool is_prime(u64 n) {
    if (n < 2) return false;
    static const u64 small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (u64 p : small)
        if (n % p == 0) return n == p;
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) {
        d >>= 1;
        ++s;
    }
    for (u64 a : small) {
        u64 x = powmod_h(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int r = 1; r < s && witness; ++r) {
            x = mulmod_h(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

// Primes q = 1 mod 2N scanned downwards from 2^bits, skipping those already
// taken: q_0 from q0_bits, then n_mid from mid_bits, then n_special from
// special_bits.  out: q_0..q_L, p_0..p_{nP-1}.
int choose_primes(int logN, int q0_bits, int n_mid, int mid_bits, int n_special, int special_bits,
                  u64 *out) {
    const u64 step = 2ull << logN;
    int n = 0;
    auto take = [&](int bits, int count) {
        u64 c = (1ull << bits) + 1 - step;
        for (int got = 0; got < count; c -= step) {
            if (c < (1ull << (bits - 1))) return false;
            if (!is_prime(c)) continue;
            bool used = false;
            for (int i = 0; i < n; ++i) used |= (out[i] == c);
            if (used) continue;
            out[n++] = c;
            ++got;
        }
        return true;
    };
    if (!take(q0_bits, 1) || !take(mid_bits, n_mid) || !take(special_bits, n_special)) return -1;
    return n;
}

u64 primitive_2n_root(u64 q, int N) {
    const u64 two_n = 2ull * (u64)N;
    for (u64 g = 2;; ++g) {
        u64 r = powmod_h(g, (q - 1) / two_n, q);
        if (powmod_h(r, (u64)N, q) == q - 1) return r;
    }
}

ModConst make_modconst(u64 q, int N) {
    ModConst m;
    m.q = q;
    m.mu = (u64)(((unsigned __int128)1 << 64) / q);
    // -q^-1 mod 2^64 by Newton iteration on the odd q
    u64 inv = q;  // correct to 3 bits
    for (int i = 0; i < 6; ++i) inv *= 2 - q * inv;
    m.qinv_neg = (u64)0 - inv;
    m.r64 = (u64)(((unsigned __int128)1 << 64) % q);
    m.r64_sh = shoup_companion(m.r64, q);
    m.r128 = mulmod_h(m.r64, m.r64, q);
    m.ninv = invmod_h((u64)N % q, q);
    m.ninv_sh = shoup_companion(m.ninv, q);
    return m;
}

// Cumulative table of |e| for the discrete Gaussian exp(-x^2 / (2 sigma^2)),
// sigma = 3.2, |x| <= 19, scaled to 2^63 (P(|e| = 0) = rho(0)/S,
// P(|e| = t) = 2 rho(t)/S).  The FP64 operation order is fixed by the
// sampler's definition and kept as written here.
void gauss_cdt(u64 cdt[20]) {
    double rho[20];
    for (int t = 0; t < 20; ++t) rho[t] = std::exp(-(double)(t * t) / (2.0 * 3.2 * 3.2));
    double total = rho[0];
    for (int t = 1; t < 20; ++t) total += 2.0 * rho[t];
    double acc = 0.0;
    for (int t = 0; t < 20; ++t) {
        acc += (t == 0 ? rho[0] : 2.0 * rho[t]) / total;
        cdt[t] = (t == 19) ? (1ull << 63) : (u64)std::ldexp(acc, 63);
    }
}

// left rotation by `rot` slots <-> X -> X^(5^rot mod 2N)
u64 galois_element(int N, int rot) {
    const int half = N / 2;
    int r = ((rot % half) + half) % half;
    u64 g = 1, two_n = 2ull * (u64)N;
    for (int i = 0; i < r; ++i) g = (g * 5) % two_n;
    return g;
}

int ext_limbs(const fr_ctx *c, int level) { return level + 1 + c->nP; }
int num_digits(const fr_ctx *c, int level) { return (level + 1 + c->alpha - 1) / c->alpha; }

}  // namespace frh
