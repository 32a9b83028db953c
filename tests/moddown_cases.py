"""Adversarial inputs for ModDown's rounding (test input builder, no method
arithmetic beyond Python-integer residues).

ModDown divides an integer U over Q_l U P by P with rounding to the nearest
integer.  The fast base conversion from the P limbs forms
X = sum_j y_j (P / p_j) with y_j = [U (P / p_j)^-1]_{p_j}, so X = (U mod P)
+ k P for a small k, and the rounding needs the integer e = round(X / P).
Coefficients whose residue U mod P sits at (P -+ 1)/2, or within a relative
2^-40 of P/2, put X / P next to a half-integer, where an FP64 estimate of
sum_j y_j / p_j cannot decide e.
"""
from __future__ import annotations

import math

import numpy as np


def residue_offsets(P: int, n: int, rng: np.random.Generator):
    """n values r = U mod P: (P-1)/2 - d and (P+1)/2 + d for small d, and
    values either side of P/2 +- P 2^-40 (the band of the exact decision)."""
    half_lo, half_hi = (P - 1) // 2, (P + 1) // 2
    band = P >> 40
    out = []
    for d in range(n // 4):
        out += [half_lo - d, half_hi + d]
    while len(out) < n:
        d = int(rng.integers(-8, 9))
        out.append(half_lo - band + d if len(out) % 2 else half_hi + band + d)
    return out[:n]


def build_u(ctx_moduli, level: int, L: int, nP: int, N: int, n_adv: int, seed: int):
    """[2][level+1+nP][N] residues of integers U = P w + r (r from
    residue_offsets on the first n_adv coefficients of each polynomial,
    uniform in [0, P) elsewhere; w uniform below Q_level) and those integers."""
    ext = list(range(level + 1)) + [L + 1 + j for j in range(nP)]
    mods = [ctx_moduli[g] for g in ext]
    P = math.prod(ctx_moduli[L + 1 + j] for j in range(nP))
    Ql = math.prod(ctx_moduli[: level + 1])
    rng = np.random.default_rng(seed)
    u = np.zeros((2, len(mods), N), dtype=np.uint64)
    Us = []
    for p in range(2):
        rs = residue_offsets(P, n_adv, rng)
        row = []
        for k in range(N):
            w = int(rng.integers(0, 2 ** 62)) * int(rng.integers(0, 2 ** 62)) % Ql
            r = rs[k] if k < n_adv else int(rng.integers(0, 2 ** 62)) * int(rng.integers(0, 2 ** 62)) % P
            U = P * w + r
            row.append(U)
            for pos, m in enumerate(mods):
                u[p, pos, k] = U % m
        Us.append(row)
    return u, Us, P


def fp64_rule_differs(u_poly, ctx_moduli, level: int, L: int, nP: int) -> int:
    """How many coefficients of one polynomial the FP64 estimate
    rint(sum_j fl(y_j) fl(1/p_j)) (summed in order, no contraction) rounds
    differently from the exact rule: the coverage of the adversarial inputs."""
    ps = [ctx_moduli[L + 1 + j] for j in range(nP)]
    P = math.prod(ps)
    phat = [P // pj for pj in ps]
    pinv = [pow(ph % pj, -1, pj) for ph, pj in zip(phat, ps)]
    n = 0
    for k in range(u_poly.shape[1]):
        s = 0.0
        X = 0
        for j, pj in enumerate(ps):
            y = int(u_poly[level + 1 + j][k]) * pinv[j] % pj
            s = s + float(y) * (1.0 / float(pj))
            X += y * phat[j]
        exact = (2 * X + P) // (2 * P)
        n += int(round(s) != exact)  # round(): nearest, ties to even, as rint
    return n
