"""Pure-Python big-integer references used to pin the C oracle.

Each function is the textbook definition, written with Python integers, and
shares nothing with the oracle's C code.
"""
import random


def negacyclic_schoolbook(a, b, q):
    """c = a * b in Z_q[X]/(X^N + 1), by the schoolbook double sum."""
    N = len(a)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                c[k] += a[i] * b[j]
            else:
                c[k - N] -= a[i] * b[j]
    return [x % q for x in c]


def crt(residues, moduli):
    """The unique X in [0, prod(moduli)) with X = r_i mod m_i (Garner-free
    formula with explicit inverses)."""
    M = 1
    for m in moduli:
        M *= m
    X = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        X += int(r) * Mi * pow(Mi, -1, m)
    return X % M


def centered(x, M):
    x %= M
    return x - M if x > M // 2 else x


def probable_prime(n, rounds=40, seed=12345):
    """Miller-Rabin with random bases (independent of the oracle's fixed bases)."""
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rnd = random.Random(seed ^ n)
    for _ in range(rounds):
        a = rnd.randrange(2, n - 1)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True
