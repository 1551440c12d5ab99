"""Search for further members of the xorgens family (test infrastructure).

Section 1.5 of arXiv:1108.0486: the family has period 2^n - 1 for n = r w
any power of two up to 4096; Section 2 adds, for the GPU, s = r/2 +- 1 with
gcd(r, s) = 1 so that min(s, r - s) terms can be computed at once.  This
script fixes (w, r, s) and looks for shift quadruples (a, b, c, d) whose
x-part has a primitive characteristic polynomial, using the oracle's GF(2)
toolkit only:

  1. P = minimal polynomial of one output bit of the x-part (Berlekamp-Massey
     on 2n + 64 bits).  If P is primitive of degree n it is the characteristic
     polynomial; a lower degree proves the candidate reducible.
  2. The primitivity test of gf2.c with the prime factors of 2^n - 1
     (Fermat numbers F_0 .. F_{log2 n - 1}).

The paper defers the quality criteria used to pick among primitive
candidates to the xorgens papers.  The reading here: shifts restricted to
[w/4, 3w/4], candidates visited in a seeded random order, the first `want`
primitive ones collected, and the one whose characteristic polynomial has
weight (number of non-zero coefficients) closest to n/2 chosen.

Usage: python -m oracle.family_search --w 64 --r 64 --s 33 [--want 4]
"""
from __future__ import annotations

import argparse
import itertools
import multiprocessing as mp
import time

import numpy as np

from oracle import fermat
from oracle import oracle as O


def member(w: int, r: int, s: int, a: int, b: int, c: int, d: int) -> O.Params:
    return O.Params(w=w, r=r, s=s, a=a, b=b, c=c, d=d, gamma=w // 2, omega=O.weyl_omega(w))


def _mersenne_factors(n: int) -> list[int]:
    m = n.bit_length() - 1
    if 1 << m != n or m > 12:
        raise ValueError("n must be a power of two up to 4096")
    return fermat.mersenne_2pow_prime_factors(m)


def check(args) -> tuple[tuple[int, int, int, int], int, int]:
    """(shifts, primitivity code, weight of P); code -1 when the minimal
    polynomial's degree is below n."""
    w, r, s, shifts = args
    p = member(w, r, s, *shifts)
    P = O.charpoly(p)
    if P.bit_length() - 1 != p.n:
        return shifts, -1, 0
    return shifts, O.is_primitive(P, _mersenne_factors(p.n)), bin(P).count("1")


def search(w: int, r: int, s: int, want: int = 4, seed: int = 1, workers: int = 8, limit: int = 200_000):
    lo, hi = w // 4, 3 * w // 4
    cands = list(itertools.product(range(lo, hi + 1), repeat=4))
    order = np.random.default_rng(seed).permutation(len(cands))[:limit]
    found, tried = [], 0
    with mp.Pool(workers) as pool:
        for shifts, code, weight in pool.imap(check, ((w, r, s, cands[i]) for i in order), chunksize=16):
            tried += 1
            if code == 0:
                found.append((shifts, weight))
                print("primitive", shifts, "weight", weight, "after", tried, flush=True)
                if len(found) >= want:
                    pool.terminate()
                    break
    n = w * r
    best = min(found, key=lambda f: abs(f[1] - n / 2)) if found else None
    return best, found, tried


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--w", type=int, required=True)
    ap.add_argument("--r", type=int, required=True)
    ap.add_argument("--s", type=int, required=True)
    ap.add_argument("--want", type=int, default=4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=8)
    a = ap.parse_args()
    t0 = time.time()
    best, found, tried = search(a.w, a.r, a.s, a.want, a.seed, a.workers)
    print("tried %d candidates in %.0f s" % (tried, time.time() - t0))
    print("chosen (a, b, c, d) =", best)


if __name__ == "__main__":
    main()
