"""Distinct prime factors of 2^4096 - 1, for the primitivity test of the
degree-4096 characteristic polynomial of the paper's xorgens member.

TEST INFRASTRUCTURE ONLY (used by tests/).

2^{2^m} - 1 = F_0 F_1 ... F_{m-1} with the Fermat numbers F_k = 2^{2^k} + 1
(since 2^{2^m} - 1 = (2^{2^{m-1}} - 1)(2^{2^{m-1}} + 1)).  For m = 12 this is
F_0 .. F_11.  F_0 .. F_4 are prime; the complete factorisations of F_5 .. F_11
are classical results of number theory (Euler; Landry and Le Lasseur;
Morrison and Brillhart; Brent and Pollard; Lenstra, Manasse et al.; Brent).
Only the small factors are listed: each large cofactor is obtained by exact
division, and the tests check every factor with a Miller-Rabin test and check
that the product is exactly 2^4096 - 1.
"""
from __future__ import annotations

# Known small prime factors of F_k; for k >= 8 one large prime cofactor remains.
SMALL_FACTORS = {
    5: [641],
    6: [274177],
    7: [59649589127497217],
    8: [1238926361552897],
    9: [2424833, 7455602825647884208337395736200454918783366342657],
    10: [45592577, 6487031809, 4659775785220018543264560743076778192897],
    11: [319489, 974849, 167988556341760475137, 3560841906445833920513],
}


def fermat(k: int) -> int:
    return 2 ** (2 ** k) + 1


def fermat_prime_factors(k: int) -> list[int]:
    F = fermat(k)
    if k <= 4:
        return [F]
    out = []
    rest = F
    for q in SMALL_FACTORS[k]:
        if rest % q:
            raise ValueError("listed factor %d does not divide F_%d" % (q, k))
        rest //= q
        out.append(q)
    if rest > 1:
        out.append(rest)
    return out


def mersenne_2pow_prime_factors(m: int = 12) -> list[int]:
    """Distinct prime factors of 2^{2^m} - 1 (m <= 12)."""
    out = []
    for k in range(m):
        out.extend(fermat_prime_factors(k))
    return out


def miller_rabin(n: int, rounds: int = 24) -> bool:
    """Probabilistic primality (deterministic bases for small n, then fixed
    pseudo-random bases)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    bases = list(small)
    x = 0x9E3779B97F4A7C15
    for _ in range(rounds):
        x = (x * 6364136223846793005 + 1442695040888963407) % 2**64
        bases.append(2 + x % (n - 3))
    for a in bases:
        a %= n
        if a < 2:
            continue
        y = pow(a, d, n)
        if y in (1, n - 1):
            continue
        for _ in range(s - 1):
            y = y * y % n
            if y == n - 1:
                break
        else:
            return False
    return True
