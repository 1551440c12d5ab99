"""Pins of the 64-bit-word oracle (xorgens64_oracle.c) and of the further
family members.

Section 1.5 of arXiv:1108.0486: the family has period 2^n - 1 for n = r w a
power of two up to 4096.  Section 2: for the GPU, s = r/2 +- 1.  The paper
gives no shifts for other members, so each member used here is pinned by the
primitivity of its characteristic polynomial (a mis-implemented shift, lag
or word size is very unlikely to stay primitive), and the 64-bit oracle's
arithmetic by an independent pure-Python generator, GF(2) linearity, the
Weyl closed form, jump-ahead against stepping, the SplitMix64 seeding and
the exact f64 mapping.
"""
import math

import numpy as np
import pytest

from oracle import fermat as F
from oracle import oracle as O

M64 = (1 << 64) - 1
W64 = O.W64


@pytest.fixture(scope="module")
def w64_poly():
    P = O.charpoly(W64)
    assert P.bit_length() - 1 == 4096
    return P


def test_w64_member_is_primitive(w64_poly):
    """(w, r, s, a, b, c, d) = (64, 64, 33, 24, 22, 37, 45): degree 4096 and
    primitive, so the x-part has period 2^4096 - 1 and with the Weyl term
    (period 2^64) the generator has period (2^4096 - 1) 2^64."""
    assert O.is_primitive(w64_poly, F.mersenne_2pow_prime_factors(12)) == 0
    ring = np.random.default_rng(3).integers(0, 2**63, size=64, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    assert O.charpoly(W64, ring=ring, bit=63) == w64_poly


def test_w64_constants():
    """omega: odd integer nearest 2^63 (sqrt 5 - 1); gamma = w / 2; s = r/2 + 1
    and gcd(r, s) = 1 (Section 2)."""
    assert O.weyl_omega(64) == W64.omega == 0x9E3779B97F4A7C15
    exact = (math.isqrt(5 * 4**63 * 4**20) - 2**63 * 2**20) / 2**20
    assert abs(W64.omega - exact) < 1.0 and W64.omega % 2 == 1
    assert W64.gamma == 32 and W64.s == W64.r // 2 + 1 and math.gcd(W64.r, W64.s) == 1


def _py_generator(ring, weyl, n, p=W64):
    """Independent pure-Python xorgens with 64-bit words: x_k from x_{k-r}
    and x_{k-s}, then Eq. (1)."""
    x = [int(v) for v in ring]
    w = int(weyl)
    out, xs = [], []
    for _ in range(n):
        t = x[-p.r]
        t ^= (t << p.a) & M64
        t ^= t >> p.b
        v = x[-p.s]
        v ^= (v << p.c) & M64
        v ^= v >> p.d
        xk = t ^ v
        x.append(xk)
        w = (w + p.omega) & M64
        out.append((xk + (w ^ (w >> p.gamma))) & M64)
        xs.append(xk)
    return out, xs


def test_w64_oracle_equals_pure_python():
    st = O.OracleStreams64(42, 2, W64)
    ring, weyl = st.ring.copy(), st.weyl.copy()
    got = st.u64(700)
    for i in range(2):
        want, _ = _py_generator(ring[i], weyl[i], 700)
        assert [int(v) for v in got[i]] == want


@pytest.mark.parametrize("kw", [dict(s=31), dict(s=32), dict(a=23), dict(d=46), dict(a=22, b=24)])
def test_w64_misreadings_are_not_primitive(kw):
    """A lag or a shift off by one, or a transposed pair, loses primitivity."""
    p = O.Params(**{**W64.__dict__, **kw})
    P = O.charpoly(p)
    if P.bit_length() - 1 == 4096:
        assert O.is_primitive(P, F.mersenne_2pow_prime_factors(12)) != 0


def test_w64_xpart_linearity():
    rng = np.random.default_rng(2)
    s1 = rng.integers(0, 2**63, size=64, dtype=np.uint64) * np.uint64(2)
    s2 = rng.integers(0, 2**63, size=64, dtype=np.uint64) * np.uint64(3)
    a, _ = O.xpart_run(W64, s1.copy(), 777)
    b, _ = O.xpart_run(W64, s2.copy(), 777)
    c, _ = O.xpart_run(W64, s1 ^ s2, 777)
    assert (c == (a ^ b)).all()


def test_w64_weyl_closed_form():
    """out_k - x_k = W_k xor (W_k >> 32) mod 2^64, W_k = W_{-1} + (k+1) omega."""
    st = O.OracleStreams64(9, 1, W64)
    ring0, w0 = st.ring[0].copy(), int(st.weyl[0])
    n = 3000
    out = st.u64(n)[0]
    # x_k from a second oracle stream with the same ring and a zero Weyl
    # start, subtracting its own (known) Weyl term
    z = O.OracleStreams64.from_state(ring0, [0], [0], W64)
    zo = z.u64(n)[0]
    k = np.arange(n, dtype=object)
    Wz = [((int(i) + 1) * W64.omega) & M64 for i in k]
    x = [(int(zo[i]) - (Wz[i] ^ (Wz[i] >> 32))) & M64 for i in range(n)]
    W = [(w0 + (int(i) + 1) * W64.omega) & M64 for i in k]
    assert all(((int(out[i]) - x[i]) & M64) == (W[i] ^ (W[i] >> 32)) for i in range(n))
    assert int(st.weyl[0]) == (w0 + n * W64.omega) & M64 and int(st.pos[0]) == n
    # and x_k is the x-part alone
    ring, _ = O.xpart_run(W64, ring0.copy(), n)
    assert int(ring[-1]) == x[-1]


@pytest.mark.parametrize("J", [1, 33, 64, 4096, 10**5])
def test_w64_jump_poly_equals_stepping(w64_poly, J):
    ring = O.OracleStreams64(5, 1, W64).ring[0].copy()
    stepped, _ = O.xpart_run(W64, ring.copy(), J)
    g = O.z_pow_mod(J, w64_poly)
    assert (O.xpart_jump_poly(W64, ring, O.poly_to_words(g, 64)) == stepped).all()


def test_w64_seeding_reading():
    """Ring and Weyl start are the first r + 1 SplitMix64 outputs of the seed
    (all 64 bits), then 4r steps are discarded; stream i uses seed + i."""
    seed = 1234
    vals = O.splitmix64_sequence(seed, 65)
    pre = O.OracleStreams64.from_state(np.array(vals[:64], dtype=np.uint64), [vals[64]], [0], W64)
    pre.skip(4 * 64)
    st = O.OracleStreams64(seed, 3, W64)
    assert (st.ring[0] == pre.ring[0]).all() and st.weyl[0] == pre.weyl[0] and st.pos[0] == 0
    assert (O.OracleStreams64(seed + 2, 1, W64).ring[0] == st.ring[2]).all()
    assert (O.OracleStreams64(seed, 1, W64, first=1).ring[0] == st.ring[1]).all()


def test_w64_f64_mapping_exact():
    a = O.OracleStreams64(42, 3, W64)
    b = a.copy()
    u = a.u64(4096)
    f = b.f64(4096)
    want = (u >> np.uint64(11)).astype(np.float64) * 2.0**-53    # 53-bit integers convert exactly
    assert (f == want).all() and f.min() >= 0.0 and f.max() < 1.0
    assert (a.ring == b.ring).all() and (a.pos == b.pos).all()


def test_r64_member_is_primitive():
    """(w, r, s, a, b, c, d) = (32, 64, 33, 19, 19, 9, 18): degree 2048 and
    primitive (2^2048 - 1 = F_0 ... F_10), with s = r/2 + 1; lag or shift
    misreadings are not."""
    p = O.R64
    assert p.s == p.r // 2 + 1 and math.gcd(p.r, p.s) == 1 and p.omega == O.PAPER.omega and p.gamma == 16
    P = O.charpoly(p)
    assert P.bit_length() - 1 == 2048
    assert O.is_primitive(P, F.mersenne_2pow_prime_factors(11)) == 0
    for kw in (dict(s=31), dict(s=35), dict(a=18), dict(c=10), dict(a=9, c=19)):
        Q = O.charpoly(O.Params(**{**p.__dict__, **kw}))
        if Q.bit_length() - 1 == 2048:
            assert O.is_primitive(Q, F.mersenne_2pow_prime_factors(11)) != 0


def test_r64_oracle_equals_pure_python():
    """The 32-bit oracle run with r = 64 against an independent pure-Python
    generator of the same member."""
    st = O.OracleStreams(42, 2, params=O.R64)
    ring, weyl = st.ring.copy(), st.weyl.copy()
    got = st.u32(500)
    p = O.R64
    for i in range(2):
        x = [int(v) for v in ring[i]]
        w = int(weyl[i])
        for t in range(500):
            a = x[-p.r]
            a ^= (a << p.a) & 0xFFFFFFFF
            a ^= a >> p.b
            v = x[-p.s]
            v ^= (v << p.c) & 0xFFFFFFFF
            v ^= v >> p.d
            x.append(a ^ v)
            w = (w + p.omega) & 0xFFFFFFFF
            assert int(got[i, t]) == ((a ^ v) + (w ^ (w >> 16))) & 0xFFFFFFFF


def test_w64_split_call_and_threads():
    a = O.OracleStreams64(42, 5, W64)
    b = a.copy()
    whole = a.u64(1001, threads=1)
    parts = np.concatenate([b.u64(500, threads=3), b.u64(1, threads=2), b.u64(500, threads=5)], axis=1)
    assert (whole == parts).all() and (a.ring == b.ring).all() and (a.weyl == b.weyl).all()


# ---- FP64 normals of the 64-bit member (the 32-bit member's Box-Muller
# pairing with 53-bit uniforms, evaluated in long double) ----

def _u1(e):
    return ((e >> 11) + 1) * 2.0**-53


def test_w64_box_muller_special_values():
    """u1 = 1 gives two zeros; u2 = 0, 1/4, 1/2, 3/4 put the whole radius on
    one axis with the right sign and an exact zero on the other; the radius
    is sqrt(-2 ln u1) (to double rounding)."""
    top = (2**53 - 1) << 11                       # (e >> 11) + 1 = 2^53: u1 = 1
    assert O.box_muller_w64(top, 12345 << 11) == (0.0, 0.0)
    for e in (0, 1 << 11, 0x0123456789ABCDEF, (2**52) << 11, M64):
        rho = math.sqrt(-2.0 * math.log(_u1(e)))
        for k, (c, s) in enumerate([(1, 0), (0, 1), (-1, 0), (0, -1)]):
            o = (k << 62) | 0x7FF                  # u2 = k / 4 (low 11 bits ignored)
            z0, z1 = O.box_muller_w64(e, o)
            for z, axis in ((z0, c), (z1, s)):
                if axis == 0:
                    assert z == 0.0, (e, k)
                else:
                    assert abs(z - axis * rho) <= 2e-16 * rho, (e, k)


def test_w64_box_muller_invariants():
    """For random pairs: z0^2 + z1^2 = -2 ln u1 and atan2(z1, z0) = 2 pi u2
    (mod 2 pi), so a dropped factor, a swapped or mis-signed branch, or a
    wrong shift of either word shows."""
    rng = np.random.default_rng(64)
    for e, o in rng.integers(0, 2**63, size=(400, 2), dtype=np.int64).tolist():
        e, o = (e << 1) | (e & 1), (o << 1) | 1
        z0, z1 = O.box_muller_w64(e, o)
        r2 = -2.0 * math.log(_u1(e))
        assert abs(z0 * z0 + z1 * z1 - r2) <= 1e-14 * max(r2, 1e-300) + 1e-300, (e, o)
        u2 = (o >> 11) * 2.0**-53
        d = (math.atan2(z1, z0) - 2 * math.pi * u2) % (2 * math.pi)
        assert min(d, 2 * math.pi - d) <= 1e-12, (e, o)


@pytest.mark.parametrize("n", [1, 2, 7, 64, 129])
def test_w64_normals_pair_consecutive_words(n):
    """The stream method pairs consecutive outputs of the call and consumes
    2 ceil(n / 2) words: it equals the pair map on a copy's u64 outputs, and
    both copies end at the same state."""
    a = O.OracleStreams64(9, 3, W64)
    b = a.copy()
    z = a.normal(n)
    w = b.u64(2 * ((n + 1) // 2))
    for i in range(3):
        want = [v for m in range(0, n, 2) for v in O.box_muller_w64(int(w[i, m]), int(w[i, m + 1]))][:n]
        assert np.array_equal(z[i], np.array(want)), i
    assert (a.ring == b.ring).all() and (a.weyl == b.weyl).all() and (a.pos == b.pos).all()


def test_w64_normals_moments():
    z = O.OracleStreams64(42, 8, W64).normal(1 << 15).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs((z**4).mean() - 3.0) < 5 * math.sqrt(96.0 / n)


@pytest.mark.parametrize("n", [1, 2, 7, 1000])
def test_w64_moments_are_the_sums_of_the_normals(n):
    """The moments kind sums exactly the normals the normal kind returns (and
    consumes the same words): against numpy sums of normal(n) to a few ulp."""
    a = O.OracleStreams64(17, 4, W64)
    b = a.copy()
    m = a.moments(n)
    z = b.normal(n)
    assert np.allclose(m[:, 0], z.sum(axis=1), rtol=0, atol=1e-12 * np.abs(z).sum(axis=1).max())
    assert np.allclose(m[:, 1], (z * z).sum(axis=1), rtol=1e-13)
    assert np.allclose(m[:, 2], np.abs(z).sum(axis=1), rtol=1e-13)
    assert (a.ring == b.ring).all() and (a.pos == b.pos).all() and (a.weyl == b.weyl).all()
